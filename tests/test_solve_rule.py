"""The host rule ucac_solve applies after each chunk of step-mode iterations
(csrc/ucac_solve_rule.hpp), compiled with the host compiler alone: the tolerance is
examined before the non-finite flag, so a chunk that reached the tolerance and went
non-finite only afterwards is replayed up to its stopping iteration (the iterations
after it never count), and the replay length puts the stop at the recorded iteration
at the chunk's first and last iterations too."""
import os
import shutil
import subprocess

import pytest

CSRC = os.path.join(os.path.dirname(__file__), "..", "paper_2310_13145_amd", "csrc")

PROGRAM = r"""
#include <cstdio>
#include "ucac_solve_rule.hpp"
int main() {
  const int cases[][3] = {{40, 1, 32}, {40, 0, 32}, {33, 1, 32}, {64, 0, 32}, {-1, 1, 32}, {-1, 0, 0}, {1, 0, 0}};
  for (const auto& c : cases) {
    const ucac::ChunkAction a = ucac::chunk_action(c[0], c[1], c[2]);
    std::printf("%d %d %d %d %d\n", c[0], c[1], c[2], (int)a.next, a.replay);
  }
  return 0;
}
"""


def test_chunk_rule(tmp_path):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    src = tmp_path / "rule.cpp"
    src.write_text(PROGRAM)
    exe = tmp_path / "rule"
    subprocess.run([cxx, "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    rows = [tuple(map(int, l.split())) for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                                check=True).stdout.split("\n") if l]
    CONTINUE, REPLAY, NONFINITE = 0, 1, 2
    expect = {
        (40, 1, 32): (REPLAY, 7),    # tolerance at the chunk's 8th iteration, non-finite later: replay, no error
        (40, 0, 32): (REPLAY, 7),
        (33, 1, 32): (REPLAY, 0),    # at the chunk's first iteration: no step-mode iteration before it
        (64, 0, 32): (REPLAY, 31),   # at its last (a chunk of 32)
        (-1, 1, 32): (NONFINITE, 0),
        (-1, 0, 0): (CONTINUE, 0),
        (1, 0, 0): (REPLAY, 0),
    }
    assert len(rows) == len(expect)
    for c0, c1, c2, nxt, rep in rows:
        assert expect[(c0, c1, c2)] == (nxt, rep), (c0, c1, c2, nxt, rep)
