// Launch interfaces between the C ABI (api.cpp) and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace kpme {

enum { PREC_FP64 = 0, PREC_FP32 = 1, PREC_BF16X3 = 2, PREC_FP16X3 = 3 };

constexpr size_t kMaxLds = 160 * 1024;  // LDS per workgroup on gfx950
constexpr int kSumBlocks = 256;          // blocks of the fixed-order FP64 sums
                                          // (scratch needs 3 * kSumBlocks doubles)

// Everything the SKP apply needs.  Pointers are device pointers; [0] is the
// single plane (FP64/FP32) or the hi plane (BF16X3), [1] the lo plane.
struct SkpArgs {
  int prec;
  int K[3];
  int K1P, K2P, K3P;     // padded extents (multiples of 32)
  int r0, R, nparts;
  int s1_split;          // split stage 1: workgroups per 64-position tile
  const void* Q;         // grid_in  [K1][K2][K3]
  void* Phi;             // grid_out [K1][K2][K3]
  const void* vec;       // split paths: per-term circulant vector copies (see stage 2)
  int blen, alen;        // lengths of one B / A vector copy (halves)
  const void* A[2];      // [R][K1P][K1P], omega folded in
  const void* B[2];      // [R][K2P][K2P]
  const void* C[2];      // [r0][K3][K3P]
  void* Y[2];            // [r0][K3][K1P][K2P]
  void* Phi_part;        // [nparts][K3][K1][K2]
  const int* term_group; // [R] group of each term (terms sorted by group)
  const int* part_begin; // [nparts + 1]
  // split-precision stage 2: steps of x3_streams terms of one group
  int x3_streams;
  const int* step_term;  // [nsteps * x3_streams], -1 = idle stream
  const int* step_group; // [nsteps]
  const int* step_begin; // [nparts + 1]
  double* scratch;       // >= kSumBlocks doubles
  // split precisions: stage 1 reduces these (sum, max) pairs into sumQ
  const double* sum_part;
  int sum_np;
  // energy from the grid (may be NULL): finalize writes, per workgroup, the
  // FP64 sum of eQ * Phi over the values it stores (finalize_blocks() of them)
  const void* eQ;
  double* epart;
  double* sumQ;          // 2 doubles: sum(Q), then the FP16X3 grid scale
  double c0;             // theta_hat_R(0)
  float sy, st;          // FP16X3 powers of two applied to Y and T before splits
  double const_scale;    // FP16X3: product of the plan-time scales
};

// LDS banks on gfx950, as measured for ds_read_b128 with the SQ bank-conflict
// counter: 64 four-byte banks (16 chunks of 16 bytes); an instruction takes
// four cycles, and the 16 lanes served in one cycle are those with equal
// (bit2 ^ bit3 ^ bit4, bit5) of the lane id.  Two of them reading different
// chunks of one bank conflict.  The layouts below are conflict-free for
// every stage-2 fragment read under this rule.
//
// Lengths of one shifted copy of the reversed circulant vectors (split
// precisions).  The copies are unwrapped over twice the padded extent, so a
// fragment's start needs no reduction modulo K and every fragment offset is
// a per-lane base plus a compile-time constant.  Lengths are multiples of 8
// halves (every copy starts 16-byte aligned); the B length is 9 chunks modulo
// 16 for every K2P (the bank offsets of the copies then follow from the
// shifts below).  The last 8 halves of a copy are never read.
inline int x3_blen(int K2P) { return 2 * K2P + 8 + (K2P % 64 == 0 ? 64 : 0); }
inline int x3_alen(int K1P) { return 2 * K1P + 16; }
// Copy s of the B vector starts x3_shift_b(s) halves past s * blen (8 for
// s = 1, 2, 7): with blen = 9 chunks mod 16 this puts the chunks that the
// lanes of one B fragment read in one cycle on distinct banks.  A copy that
// starts earlier than the previous one ends overwrites that copy's unread
// tail (the host fills the copies in order).  Copy s >= 1 of the A vector
// starts kX3ShiftA halves past s * alen.  One plane of a term:
// [B copies | A copies], 8 * blen + 8 + 4 * alen + 8 halves.
__host__ __device__ constexpr int x3_shift_b(int s) { return 8 * ((0x86 >> s) & 1); }
constexpr int kX3ShiftA = 4;
inline int x3_plane(int K1P, int K2P) { return 8 * x3_blen(K2P) + 8 + 4 * x3_alen(K1P) + 8; }
// Swizzle of the stage-2 Y slab in LDS: rows of K2P halves without padding,
// 16-byte chunk c of row r stored at chunk c ^ x3_yswz(NKC, r) (NKC = K2P / 32;
// the XOR stays inside the row).
__host__ __device__ constexpr int x3_yswz(int NKC, int r) {
  return NKC == 4 ? (r & 15) : NKC == 2 ? ((r >> 1) & 7) : ((r >> 1) & 3);
}
// Split-precision stage 2 shape: column tiles of 16 per wave (CT) and term
// streams per workgroup (NS, 1 or 2: every stream has its own waves over the
// shared Y slab, so NS sets the waves per workgroup).  96 x 96 slabs: two
// streams of two 48-column waves (four-wave workgroups, two per CU: two waves
// on every SIMD).  x3_streams is the default; the autotuner times both.
constexpr int x3_ct(int K1P, int K2P) { return (K1P == 96 && K2P == 96) ? 3 : 2; }
constexpr int x3_streams(int K1P, int K2P) { return ((K1P == 96 && K2P == 96) || (K1P == 128 && K2P == 128)) ? 2 : 1; }

hipError_t launch_skp_sum(const SkpArgs& a, hipStream_t st);
// the per-block (sum, max) pairs of launch_skp_sum only, into a.scratch
hipError_t launch_sum_partials(const SkpArgs& a, hipStream_t st);
hipError_t launch_skp_stage1(const SkpArgs& a, hipStream_t st);
hipError_t launch_skp_stage2(const SkpArgs& a, hipStream_t st);
// Raises the dynamic-LDS limit of the stage-2 kernel instance that `a`
// selects; called once at plan creation, so that no attribute change is ever
// issued between launches (or inside a stream capture).
hipError_t prepare_skp_stage2(const SkpArgs& a);
hipError_t launch_skp_finalize(const SkpArgs& a, hipStream_t st);
size_t stage2_lds_bytes(int prec, int K1P, int K2P, int streams);

// Grid kernels: binning, spread and gather.

struct GridGeom {
  int K[3];
  double L[3];
  double invL[3];  // 1 / L
  int p;
  // interpolation: 0 = order-p cardinal B-splines; c > 0 = per-cell Lagrange
  // interpolation on cells of c = p - 1 grid intervals (p nodes per axis,
  // end points shared with the neighbouring cells)
  int cell = 0;
};

// Record length of the per-axis neighbour table: {count, up to 4 bricks}.
constexpr int kNbrRec = 5;

// Brick decomposition of the grid used to bin particles.
struct BinGeom {
  int edge[3];   // brick edge in grid points
  int nb[3];     // bricks per axis, ceil(K / edge)
  int nbricks;
  int nbmax;     // row stride of the neighbour table
  int two_homes; // every owner brick reached by exactly two home bricks per
                 // axis (itself and the next) and every tile extent <= K_j
  int sparse;    // few particles per brick: the owner spread also for
                 // orders 4 and up on float grids
  int gather_wgs; // target workgroup count of the persistent gather (one
                  // brick per workgroup up to it)
};

// Device buffers of the binned particle layout.
struct Bins {
  BinGeom geom;
  int* count;     // [nbricks + 1] histogram
  int* offset;    // [nbricks + 1] exclusive prefix sums
  int* brick_of;  // [max_n]
  int* slot;      // [max_n] rank inside the brick
  int* perm;      // [max_n] sorted position -> caller index
  int* nbr;       // [3][nbmax][kNbrRec] home bricks reaching each owner brick
  void* tiles;    // [nbricks][(edge + p - 1)^3] per-brick spread tiles (plan precision)
  void* sorted;   // [max_n][4] x, y, z, q in binned order (plan precision)
};

// All launches are asynchronous on `st`; they return the launch status.
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);
hipError_t launch_gather_direct(int prec, const GridGeom& g, int64_t n, const void* pos,
                                const void* q, const void* grid, void* pot, void* force,
                                hipStream_t st);
// qpart: per scatter workgroup the FP64 (sum q, sum q^2), scatter_partials()
// pairs.
hipError_t launch_bin(int prec, const GridGeom& g, const Bins& b, int64_t n, const void* pos,
                      const void* q, double* qpart, hipStream_t st);
int scatter_partials(const Bins& b, int64_t n);
int spread_partials(const BinGeom& bg, int p, bool fp64);

// Final energies of an evaluation, combined by one workgroup: E_rec = 1/2 of
// the sum of the finalize partials (sum over grid points of Q Phi, equal to
// 1/2 sum_i q_i phi_i since the B-spline weights of a particle sum to one),
// E_self = -beta / sqrt(pi) sum q^2, E_neutral = -pi (sum q)^2 / (2 V beta^2),
// their sum; e4 = NULL: nothing to do.
struct EnergyJob {
  const double* epart = nullptr;
  int nfin = 0;
  const double* qpart = nullptr;
  int nq = 0;
  double beta = 0, volume = 0;
  double* e4 = nullptr;
};
hipError_t launch_energy_job(const EnergyJob& ej, hipStream_t st);
int finalize_blocks(int K1, int K2, int K3);
// part2 (2 doubles per brick): the tile's sum and largest magnitude.  src:
// binned (x, y, z, charge) records to spread (NULL: the plan's own bins).
hipError_t launch_spread_binned(int prec, const GridGeom& g, const Bins& b, void* grid,
                                double* part2, hipStream_t st, const void* src = nullptr);
// ej.e4 != NULL: one extra workgroup of the gather runs the energy job.
hipError_t launch_gather_binned(int prec, const GridGeom& g, const Bins& b, int64_t n,
                                const void* grid, void* pot, void* force, const EnergyJob& ej,
                                hipStream_t st);
hipError_t launch_resort_charges(int prec, const Bins& b, int64_t n, const void* gval,
                                 void* sorted2, hipStream_t st);
hipError_t launch_gather_backward(int prec, const GridGeom& g, const Bins& b, int64_t n,
                                  const void* Phi, const void* Psi, const double* g_energy,
                                  const void* g_pot, const double* sumq, double beta,
                                  double volume, void* grad_pos, void* grad_q,
                                  hipStream_t st);
// Combines np (sum, max) pairs: out[0] = sum, out[1] = FP16X3 grid scale.
hipError_t launch_sum_final(const double* part2, int np, double* out, hipStream_t st);
hipError_t launch_energy(int prec, int64_t n, const void* q, const void* pot, double beta,
                         double volume, double* scratch, double* energy4, hipStream_t st);

}  // namespace kpme
