// Shared host/device definitions of the FoE + iPiano library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace foe {

constexpr int KS = 7;           // filter size
constexpr int KK = KS * KS;     // taps per filter
constexpr int R = 3;            // filter radius
constexpr int MAX_NF = 64;
constexpr int PART_COLS = 8;    // per-block partial sums: F, G, s1, s2, m, (unused) x3
constexpr int STAT_COLS = 8;

enum Model { COMBINED = 0, LOG = 1, IDIV = 2 };
enum Boundary { SYMMETRIC = 0, ZERO = 1, PERIODIC = 2 };
enum StepMode { BACKTRACK = 0, FIXED = 1 };
enum Status { ST_OK = 0, ST_ELINESEARCH = 4, ST_ENONFINITE = 5, ST_EINPUT = 6 };

// iPiano state kept in device memory; written only by the single-block decide kernel
// and by the host before a launch sequence.
struct DevState {
  double L;            // current Lipschitz estimate (of the trial being run)
  double alpha;        // current step
  double Fcur;         // F(x^n)
  double L_acc;        // L of the last accepted trial
  double sums[PART_COLS];  // totals of the last reduction
  int icur, iprev, icand;  // x ring indices: x^n, x^{n-1}, candidate
  int gcur, gcand;         // gradient ring indices: grad F(x^n), candidate grad F(x+)
  int iter;                // accepted iterations of this launch sequence
  int target;              // iterations requested
  int trials;              // trials of the current iteration so far
  int total_trials;
  int status;              // Status
  int done;                // 1 => every later trial / decide launch is a no-op
  int input_bad;           // set by the init kernel when f or u0 is invalid
  int pending;             // 1 => a trial has run whose partials await the decision
  long long t_start;       // device wall clock when the solve's initial state was written
  long long t_done;        // device wall clock of the decision that completed the image (0 while running)
};

// One image of a (possibly single-image) batch: packed-plane offset, size, data-term weights and
// its range in the tile list.
struct ImageDesc {
  long long off;
  int H, W;
  float lam1, lam2;
  int tile0, ntiles;
};

// One output tile of the flattened tile list over all images.
struct TileDesc {
  int image, x0, y0, pad;
};

// The tile (row-major index over the image's n tiles) of the image's i-th block.  Workgroups are dealt to
// the 8 XCDs in turn (block b on XCD b % 8); the blocks of one residue class i % 8 take consecutive tiles,
// so that neighbouring tiles, which read each other's halo lines, meet in one L2 (exactly so for an image
// whose first block is a multiple of 8, as in every single-image solve).  The order depends on n alone,
// so an image runs the same tile order, and sums its partials in the same order, alone or in a batch.
__host__ __device__ inline int xcd_tile_order(int i, int n) {
  const int c = i % 8, r = i / 8, q = n / 8, rem = n % 8;   // classes c < rem hold q + 1 blocks, the others q
  return c * q + (c < rem ? c : rem) + r;
}

// Solver-wide constants (shared by every image of a batch).
struct Problem {
  int H, W;
  int nf;
  int model, bc, step_mode;
  int max_backtracks, newton_iters;
  int prox_method;  // 0 Newton, 1 Lambert W (LOG model)
  int engine;  // forward-bank engine of the fused kernel
  float beta;
  double beta_d, eta_up, eta_down, alpha_fixed;
};

}  // namespace foe
