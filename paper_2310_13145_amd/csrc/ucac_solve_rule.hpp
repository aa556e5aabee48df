// What ucac_solve does after a chunk of step-mode iterations, from the control block
// it read back (host code; no device types).
//
// A step-mode control step cannot stop an instance, so it records the first iteration
// of the solve at which r_p, r_d <= tol (conv_iter, counted from 1; -1 if none) and
// raises a flag on a non-finite residual (bad).  The tolerance is examined first: a
// chunk that reached it and went non-finite only afterwards is replayed from its
// snapshot up to the stopping iteration (replay step-mode iterations, then one
// solve-mode iteration that stops the instance there), so the iterations after it
// never count; only a chunk that never reached the tolerance ends the solve on the flag.
#pragma once

namespace ucac {

enum ChunkNext { CHUNK_CONTINUE, CHUNK_REPLAY, CHUNK_NONFINITE };

struct ChunkAction {
  ChunkNext next;
  int replay;  // CHUNK_REPLAY: step-mode iterations before the stopping one
};

// launched: iterations of the solve before this chunk.
inline ChunkAction chunk_action(int conv_iter, int bad, int launched) {
  if (conv_iter > 0) return ChunkAction{CHUNK_REPLAY, conv_iter - launched - 1};
  if (bad) return ChunkAction{CHUNK_NONFINITE, 0};
  return ChunkAction{CHUNK_CONTINUE, 0};
}

}  // namespace ucac
