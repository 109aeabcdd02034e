// Internal interfaces between the host API and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qst {

// Geometry of one instance on the staged butterfly path.
//   n_lo : low qubits (index bits [0, n_lo)), handled by the fused stage with all
//          atoms on chip; R * 2^n_lo fits one work-group's LDS.
//   n_hi : high qubits (bits [n_lo, n)), handled by the tile stages A and C.
//   t, c : the tile stages hold 2^t amplitudes of one atom: 2^n_hi rows (stride
//          2^n_lo) by 2^c contiguous columns, t = n_hi + c.
//   grid_lo : work-groups of the persistent low stage (one launch per batch); each
//          takes every grid_lo-th chunk (one setting x 2^n_lo outcomes, all atoms).
//   S    : settings per batch (X and W hold S x R x D amplitudes).
struct Geometry {
  int n, R, B;
  long long D;
  int n_lo, n_hi, t, c;  // n_hi: every index bit above the low stage
  int t_adj, c_adj;  // tile of the adjoint stage C (may differ from stage A's)
  // Three-pass schedule (n_mid > 0): the bits above the low stage are more than one tile holds,
  // so index bits [n_lo, n_lo + n_mid) get a middle pass of their own (in place on X and on W,
  // tiles of 2^14 amplitudes with 2^c_mid contiguous columns) and stages A and C rotate the top
  // n_hi - n_mid bits.
  int n_mid, c_mid;
  int logv_lo;  // registers per thread in the low stage: 2^logv_lo
  int grid_lo;
  int S;
  int elem;      // bytes per real (4 or 8)
  int split_adj; // work-groups per adjoint tile at batch size S (partial-sum slices in the workspace)
  bool h16;      // the setting-batch intermediates X and W are stored in BF16
  bool gen;      // general local settings: a rotation and a phase per (setting, qubit) from the decode
  bool sparse;   // sparse (CSR) frequencies: chunk pointers in the workspace
  // Two-sweep low stage (lo2): the low stage takes n_lo = n - 10 bits with the atoms looped in
  // one work-group (X read twice), so the bits above it fit one tile pass (n_mid = 0).
  bool lo2;
};

struct LoArgs {
  const void* src;            // X [S][R][D] or the atoms [R][D]
  long long src_set_stride;   // elements between consecutive settings in src (0: atoms)
  void* dst;                  // W [S][R][D] (adjoint pass)
  const uint64_t* pc;         // decoded settings [B]
  const double* alpha;        // [R]
  const float* freqs;         // [B][D] or null
  const void* grad_p;         // [B][D] or null (generic sensitivity)
  void* probs;                // [B][D] or null
  const void* pbase;          // [B][D] or null: base probabilities added to p
  const float* um;            // general settings: [B][n][8] (tan(theta/2), sin(theta), Re e, Im e, 0...) by index bit (else null)
  // sparse frequencies (freqs then holds the non-zero values): fidx [nnz] outcomes, fchunk
  // [B * 2^n_hi + 1] the first non-zero of each (setting, high index) chunk; null: dense
  const int* fidx;
  const long long* fchunk;
  long long fnnz;
  void* gneg;                 // [B][D] or null: receives -dL/dp
  double* part;               // [(R+1)][nslots]: row 0 loss, rows 1..R weight gradient
  long long nslots;
  long long slot_base;        // first slot of this launch (batch index x grid)
  int nchunks;                // chunks of this instance: settings of the batch x 2^n_hi
  long long D;
  int R, n, n_lo, n_hi, log_ta, b0, B;
  int loss_kind;
  double eps;
  // Orders of X (input) and W (output): the top x_up (w_up) index bits of a chunk are stored
  // above the high bits, so that the tile stages' rows lie 2^(n_lo - x_up) (2^(n_lo - w_up))
  // elements apart (0: plain [S][R][D] order)
  int x_up, w_up;
};

// One launch of the low stage over several instances of the same low-bit count:
// chunks [begin[k], begin[k+1]) belong to instance a[k]; rmax is the largest rank
// (block size and LDS layout).  Passed by value, so a captured graph keeps it.
constexpr int kBatchMax = 16;
struct LoBatch {
  int count;
  int total;
  int rmax;
  int begin[kBatchMax + 1];
  LoArgs a[kBatchMax];
};
static_assert(sizeof(LoBatch) <= 4096, "kernel argument block too large");

struct HiArgs {
  const void* src;  // forward: atoms [R][D];   adjoint: W [S][R][D]
  void* dst;        // forward: X [S][R][D];    adjoint: atom gradient [R][D]
  const uint64_t* pc;
  const float* um;  // general settings: [B][n][8] (tan(theta/2), sin(theta), Re e, Im e, 0...) by index bit (else null)
  void* part;       // adjoint with nsplit > 1: per-split sums [nsplit][R][D]
  long long D;
  int R, n, n_lo, n_hi, t, c, b0, S, first;
  int nsplit;       // work-groups per tile, each over a contiguous share of the S settings
  int w_up;         // forward: the order of X (LoArgs::x_up); adjoint: of W (LoArgs::w_up)
};

// Middle pass of the three-pass schedule: index bits [row_lo, row_lo + rows) of every (setting,
// atom) vector of a batch, rotated in place (no phases).
struct MidArgs {
  void* buf;        // X (forward) or W (adjoint): [S][R][D]
  const uint64_t* pc;
  const float* um;  // general settings (else null), as in HiArgs
  long long D;
  int R, n, row_lo, rows, t, c, b0, S;
  int nsplit;       // work-groups per tile, each over a contiguous share of the S settings
};

// Batches of small instances (whole state in one low-stage chunk, all settings in
// one batch): one launch per step for up to kBatchMax instances, arguments by value.
struct DecodeBatch {
  int count;
  int total;
  int N;
  int begin[kBatchMax + 1];
  const uint8_t* settings[kBatchMax];
  uint64_t* pc[kBatchMax];
};
struct SumBatch {  // grad_k[e] = sum_s W_k[s][e], e < R_k D
  int count;
  int elem;
  int h16;  // W in BF16
  long long total;
  long long begin[kBatchMax + 1];
  const void* W[kBatchMax];
  void* grad[kBatchMax];
  long long RD[kBatchMax];
  int S[kBatchMax];
};
struct RowBatch {  // fixed-order sums of the per-work-group partials
  int count;
  int rmax;
  long long nslots;
  const double* part[kBatchMax];
  int R[kBatchMax];
  double* loss[kBatchMax];   // null: no loss row
  double* wgrad[kBatchMax];  // null: no weight-gradient rows
};
struct TanBatch {  // grad_k[r] -= psi_k[r] <psi_k[r], grad_k[r]>
  int count;
  int rmax;
  int elem;
  const void* atoms[kBatchMax];
  void* grad[kBatchMax];
  int R[kBatchMax];
  long long D[kBatchMax];
};
hipError_t launch_decode_batch(const DecodeBatch& b, int* flag, hipStream_t st);
hipError_t launch_sum_batch(const SumBatch& b, hipStream_t st);
// grad[e] (first: =, else +=) sum_{k < nsplit} part[k][e], e < RD, in order of k.
hipError_t launch_sum_splits(int elem, const void* part, int nsplit, long long RD, void* grad, int first,
                             hipStream_t st);
hipError_t launch_rowsum_batch(const RowBatch& b, hipStream_t st);
hipError_t launch_tangent_batch(const TanBatch& b, hipStream_t st);

// Launchers (return the HIP status of the launch).
hipError_t launch_decode(const uint8_t* settings, int B, int N, uint64_t* pc, int* flag, hipStream_t st);
// g: geometry of the largest rank in the batch (LDS size, grid).
hipError_t launch_stage_lo(const Geometry& g, const LoBatch& m, bool adjoint, hipStream_t st);
hipError_t launch_stage_hi(const Geometry& g, const HiArgs& a, bool adjoint, hipStream_t st);
// Middle pass (g: the instance's geometry; a.rows = g.n_mid, a.c = g.c_mid).
hipError_t launch_stage_mid(const Geometry& g, const MidArgs& a, bool adjoint, hipStream_t st);
// Two-sweep low stage (qst_lo2.hip): n_lo 10..14, FP32 Pauli settings, dense data, X and W in
// FP32 or BF16 (g.h16).
hipError_t launch_stage_lo2(const Geometry& g, const LoArgs& a, bool adjoint, hipStream_t st);
int lo2_occupancy(const Geometry& g);
size_t lo2_lds_bytes(const Geometry& g);
hipError_t launch_sum_settings(const Geometry& g, const void* W, int S, void* grad, int first, hipStream_t st);
hipError_t launch_fill(void* p, size_t bytes, hipStream_t st);
// Sparse frequencies: cptr[b * nh + h] = first non-zero of row b with outcome >= h * U
// (rows from rowptr, outcomes in idx), cptr[B * nh] = nnz; every entry clamped to [0, nnz].
hipError_t launch_chunk_ptr(const long long* rowptr, const int* idx, long long nnz, int B, int nh, int U,
                            long long* cptr, hipStream_t st);
// General local settings: per (setting, qubit) the rotation form of its 2x2 (Pauli codes
// 0..2 or unitaries[code - 3]), R = [[c, -s], [s, c]] after the input phase diag(1, e), as
// (tan(theta/2), s, Re e, Im e) at um[(b * N + index bit) * 8]; pc gets code 0 for every qubit.  Codes
// >= 3 + K OR 1 into the flag, table entries that are not unitary OR in 2 (both: identity).
hipError_t launch_decode_general(const uint8_t* settings, int B, int N, const double* unitaries, int K, float* um,
                                 uint64_t* pc, int* flag, hipStream_t st);
// part [rows][nslots] -> out[rows] (two-level, fixed order).  out_stride: spacing of out entries.
hipError_t launch_rowsum(const double* part, int rows, long long nslots, double* lvl1, int g1, double* out,
                         hipStream_t st);
// Write the reduced loss / weight gradient to the caller's buffers.
hipError_t launch_scatter_results(const double* sums, int R, double* loss, double* wgrad, hipStream_t st);
// a7: grad[r] -= psi_r <psi_r, grad[r]>  (per atom, FP64 inner products)
hipError_t launch_tangent(int elem, const void* atoms, void* grad, int R, long long D, double* scratch,
                          int g1, hipStream_t st);
hipError_t launch_reweight(const double* alpha, const double* h, int R, double eta, double tau,
                           double* alpha_out, int32_t* keep, int32_t* R_out, hipStream_t st);

// Stage the atom-step pair: pair [2][D] = (psi_trial, atoms[r]), wpair = (alpha_r, -alpha_r).
hipError_t launch_atom_pair(int elem, const void* trial, const void* atoms, const double* alpha, int r, long long D,
                            void* pair, double* wpair, hipStream_t st);

// Iteration helpers: the normalised trial atom (psi + eta d) / ||psi + eta d|| (part: kTrialBlocks
// doubles, lvl1: g1 doubles, sumsq: one double), and a row gather with zero fill.
constexpr int kTrialBlocks = 1024;
hipError_t launch_trial_atom(int elem, const void* psi, const void* d, double eta, void* y, long long D,
                             double* part, double* lvl1, int g1, double* sumsq, hipStream_t st);
hipError_t launch_gather_rows(int elem, const void* src, const int32_t* idx, const int32_t* count, int rows_max,
                              long long D, void* dst, hipStream_t st);

// Plain per-qubit reference path (FP32).
hipError_t launch_plain_copy(const void* atoms, void* X, int S, int R, long long D, hipStream_t st);
hipError_t launch_plain_qubit(void* X, int S, int R, long long D, int bit, const uint64_t* pc, int b0, bool adj,
                              hipStream_t st);
hipError_t launch_plain_point(const LoArgs& a, void* X, int S, hipStream_t st);
hipError_t launch_plain_sum(const void* X, int S, int R, long long D, void* grad, int first, hipStream_t st);

// MFMA tile path: one pass over X [S][R][D] (complex64, in place) applying the
// setting's 16x16 tile (adjoint: its conjugate transpose) on index bits [gb, gb+4).
hipError_t launch_tile_pass(void* X, int S, int R, long long D, int gb, const uint64_t* pc, int b0, bool adj,
                            bool bf16, hipStream_t st);

// Vector helpers for the refactorisation (complex128 Krylov vectors).
hipError_t launch_dots(const void* Q, int k, long long ldq, const void* w, int w_is_c64, long long D,
                       double* part, int g1, double* out_re_im, hipStream_t st);
hipError_t launch_combine(void* w, const void* Q, int k, long long ldq, const double* coef_re_im, double sign,
                          int q_is_c64, long long D, hipStream_t st);
hipError_t launch_convert(const void* src, int src_c64, void* dst, int dst_c64, long long n, double scale_re,
                          hipStream_t st);
hipError_t launch_axpy_c(void* y, int y_c64, const void* x, int x_c64, long long n, double a, hipStream_t st);

// On-chip path (qst_onchip.hip): states of 2^11 .. 2^14 amplitudes, FP32, Pauli settings,
// dense data.  One entry per instance of a call, in device memory (written by k_oc_stage
// from by-value chunks).  Pass F items: settings [j sF, (j+1) sF) of instance k; pass A items:
// slice j / ntile (settings [slice sA, (slice+1) sA)), atoms [tile VPW, (tile+1) VPW) with
// tile = j % ntile.  Loss partials go to part[0][j] (j < nF = nslots), weight-gradient
// partials to part[1+r][slice] (slices < nA <= nF; pass F zeroes the rest).
struct OcInst {
  const void* atoms;    // [R][D] complex64
  const double* alpha;  // [R]
  const uint64_t* pc;   // decoded settings [B]
  const float* freqs;   // [B][D] or null
  const float* grad_p;  // [B][D] or null: caller's dL/dp (then pass F is skipped)
  const float* pbase;   // [B][D] or null
  float* probs;         // [B][D] or null
  float* gneg;          // [B][D] or null: receives -dL/dp
  float* G;             // [B][D] workspace: 2^-k dL/dp of pass F (null with grad_p)
  float2* P;            // [nA][R][D] workspace: slice partials (unused when nA == 1)
  float2* grad;         // [R][D] atom gradient (null: forward only)
  double* part;         // [(R+1)][nslots] or null
  double* loss;         // device scalar or null
  double* wgrad;        // [R] or null
  const uint8_t* settings;  // [B][n] Pauli codes (decoded into pc_out by k_oc_decode)
  uint64_t* pc_out;         // the same array as pc
  long long nslots;
  double eps;
  int n, R, B, loss_kind;
  int sF, sA, nA, ntile;
  int itemF0, itemA0, sumB0, tangent;
  int decB0, pad;           // first block of this instance in the decode launch
};
static_assert(sizeof(OcInst) % 4 == 0, "staged as 32-bit words");
constexpr int kOcChunk = 16;
struct OcChunk {
  int count;
  int first;
  OcInst a[kOcChunk];
};
static_assert(sizeof(OcChunk) <= 4096, "kernel argument block too large");
// 2^logv values per thread (5 for n = 11..14, or 4 for n = 13, 14: twice the threads).
bool oc_shape_ok(int n, int logv);
size_t oc_lds_bytes(int n, int logv);
int oc_threads_of(int n, int logv);
int oc_blocks_per_cu(int n, int logv, bool adj);
// Pass F (adj = false) or A over items [0, total) of instances [k0, k1) (all of n qubits).
hipError_t launch_oc_pass(int n, int logv, bool adj, const OcInst* tab, int k0, int k1, int total, int grid,
                          hipStream_t st);
// Fused slices (states with R 2^n <= 2^14): items (instance, slice) as in pass A, every atom of
// a setting in one work-group of fs_threads(n, RM) threads (RM: the largest rank of the launch).
hipError_t launch_fs_pass(int n, bool adj, const OcInst* tab, int k0, int k1, int total, int RM, int grid,
                          hipStream_t st);
int fs_blocks_per_cu(int n, bool adj, int RM);
hipError_t launch_oc_stage(const OcChunk& c, OcInst* tab, hipStream_t st);
// Decode the settings of every instance of the table (blocks: sum of ceil(B / 256)).
hipError_t launch_oc_decode(const OcInst* tab, int count, int blocks, int* flag, hipStream_t st);
// Slice sums (sum_blocks > 0), loss and weight-gradient rows (rows), tangent projection.
hipError_t launch_oc_finish(const OcInst* tab, int count, int sum_blocks, int rmax, bool rows, bool tangent,
                            hipStream_t st);

// Grouped low stage of the G v products (one vector, FP32, Pauli settings, 14 low bits):
// settings that share their high-bit codes (a pattern) share stage A's output X_P and
// stage C's input W_P.  Item (pattern p0 + s, high index h): X_P's chunk h in registers,
// W_P's chunk h = sum over the members b of the pattern of
// L_b^dagger (alpha 2^-k_b g_b * L_b X_P) (L_b: the low-bit part of V_b, phases included).
struct GvArgs {
  const float2* X;      // [S][D] stage A output of patterns p0 .. p0 + S - 1
  float2* W;            // [S][D]
  const uint64_t* pc;   // [B] code words of the settings (all n qubits)
  const int* perm;      // [B] the settings ordered by pattern
  const int* goff;      // [P + 1] first position in perm of each pattern's members
  const float* g;       // [B][D] sensitivities g_b
  const double* alpha;  // [1] the vector's weight
  int n, p0, S;
};
constexpr int kGvLoBits = 14;
size_t gv_lds_bytes();
int gv_blocks_per_cu(int logv);
hipError_t launch_gv_lo(const GvArgs& a, int logv, int grid, hipStream_t st);

// Register bits per thread of the low stage (2^logv values): 5, or 4 in the forward pass
// over staged chunks of 2^12 and more outcomes (ranks up to 4: twice the wavefronts).
constexpr int lo_logv_of(int n_lo, bool staged, bool adjoint) {
  return n_lo < 5 ? n_lo : ((staged && !adjoint && n_lo >= 12) ? 4 : 5);
}
// LDS of the low stage with 2^logv values per thread; lo_lds_bytes: the larger of the
// forward and the adjoint pass.
size_t lo_lds_bytes_logv(const Geometry& g, int logv);
size_t lo_lds_bytes(const Geometry& g);
int lo_blocks_per_cu(const Geometry& g);
size_t hi_lds_bytes(const Geometry& g);

}  // namespace qst
