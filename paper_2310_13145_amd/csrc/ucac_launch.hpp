// Host-side launchers of the iteration kernels (one translation unit each).
#pragma once
#include "ucac_dev.hpp"
#include "ucac_ctl.hpp"

namespace ucac {
// the unit side (generator update, UC dynamic program, relaxed commitments) per generator
void launch_units(const Net& n, const State& s, const Par& p, hipStream_t st);
void launch_units_lanes(const Net& n, const State& s, const Par& p, hipStream_t st, int dp_lanes);
void launch_branch(const Net& n, const State& s, const Par& p, hipStream_t st);
void launch_branch_block(const Net& n, const State& s, const Par& p, hipStream_t st, int block);
// The line kernel at 256-lane blocks, timed by the dispatch's own start/stop events.
// Timed launches of the kernel-by-kernel iteration's kernels: the launch carries its
// own start and stop events (the dispatch's begin and end timestamps); false where the
// kernel has no work and nothing was launched (the events stay unrecorded).  The line
// kernel's pair does not cover the learned start's network kernel launched before it.
bool launch_units_timed(const Net& n, const State& s, const Par& p, hipStream_t st, hipEvent_t e0, hipEvent_t e1);
bool launch_branch_timed(const Net& n, const State& s, const Par& p, hipStream_t st, hipEvent_t e0, hipEvent_t e1);
bool launch_bus_timed(const Net& n, const State& s, const Par& p, hipStream_t st, hipEvent_t e0, hipEvent_t e1);
bool launch_post_timed(const Net& n, const State& s, const Par& p, hipStream_t st, hipEvent_t e0, hipEvent_t e1);
bool launch_finalize_timed(const Net& n, const State& s, const Par& p, hipStream_t st, hipEvent_t e0, hipEvent_t e1);
void launch_bus(const Net& n, const State& s, const Par& p, hipStream_t st);
void launch_post(const Net& n, const State& s, const Par& p, hipStream_t st);
void launch_finalize(const Net& n, const State& s, const Par& p, hipStream_t st);  // slots: standard_ranges(s, s.red_u)
void launch_finalize_ranges(const State& s, const Par& p, const SlotRanges& R, hipStream_t st);
void launch_lambda(const Net& n, const State& s, const Par& p, hipStream_t st);

// Blocks of each kernel's single-instance grid (what one member contributes to a
// grouped launch).  K_ITER kernels per iteration; K_LAMBDA flushes a pending
// multiplier update after a call.
// K_FRONT: the unit side and the lines in one launch (the units' and the lines' block
// tables side by side); the iteration graph runs K_FRONT, K_BUS, K_POST, K_FINALIZE.
enum { K_UNITS, K_BRANCH, K_BUS, K_POST, K_FINALIZE, K_ITER, K_LAMBDA = K_ITER, K_COUNT, K_FRONT = K_COUNT };
int units_gpb(int T, int dp_lanes, int bs);  // generators per unit block of bs threads
size_t units_lds(int T, int gpb);    // dynamic LDS of a unit block
int units_blocks(const Net& n, int gpb);
int branch_blocks(const Net& n, int block);
int bus_blocks(const Net& n);
int post_blocks(const Net& n);
int lambda_blocks(const Net& n);
// the unit side and the lines in one launch: the units' blocks first, then the lines';
// with fin_units >= 0 a first block runs the previous iteration's control step
void launch_front(const Net& n, const State& s, const Par& p, hipStream_t st, int fin_units = -1);
// The fused iteration (two launches): the finish of the previous iteration's rows
// (mode bit 1) and this iteration's unit side and lines (mode bit 2) in one launch;
// then the bus solve without rows G1, G2, with the previous iteration's control step
// over the slot ranges *fin in a first block (none if fin is null).
enum { FUSE_PRO = 1, FUSE_WORK = 2 };
void launch_front_fused(const Net& n, const State& s, const Par& p, hipStream_t st, int mode);
void launch_bus_fused(const Net& n, const State& s, const Par& p, hipStream_t st, const SlotRanges* fin);
void launch_front_grouped(const Group& gu, int grid_u, const Group& gb, int grid_b, int warm_start, int block,
                          int dp_lanes, int max_T, hipStream_t st);
void launch_bus_grouped(const Group& g, int grid, hipStream_t st);
void launch_post_grouped(const Group& g, int grid, hipStream_t st);
void launch_finalize_grouped(const Group& g, int grid, hipStream_t st);
void launch_lambda_grouped(const Group& g, int grid, hipStream_t st);

// standalone UC dynamic programs on given tables (k_units.hip)
size_t dp_tables_lds(int T, int lanes);
void launch_dp_tables(const double* tab, int G, int T, const int* tu, const int* td, const int* u0, const int* lon,
                      const int* loff, signed char* u_out, double* cost_out, int lanes, hipStream_t st);

// learned warm start (k_mlp.hip)
void mlp_launch_train(const MlpView& w, const float* X, const float* Yt, const int* idx, int nb, float inv_norm,
                      float* slots, hipStream_t st);
void mlp_launch_reduce(const float* slots, int n_slots, float* grad, double* loss, float* P, float* m1, float* m2, int step,
                       float lr, __bf16* W1b, __bf16* W2b, __bf16* W3b, hipStream_t st);
void mlp_launch_pack(const float* P, __bf16* W1b, __bf16* W2b, __bf16* W3b, hipStream_t st);
void mlp_launch_forward(const MlpView& w, const float* X, int n, float* Y, hipStream_t st);
constexpr int MLP_PARAMS = 5764;   // 64*20 + 64 + 64*64 + 64 + 4*64 + 4
constexpr int MLP_SLOT = MLP_PARAMS + 4;
}  // namespace ucac
