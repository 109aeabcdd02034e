// Small kernels of the hot path: descriptor decode, fills, the per-setting
// sums of the single-chunk geometry, deterministic reductions, the tangent
// projection, the FP64 coefficient step, the plain one-pass-per-qubit
// reference path and the vector helpers of the refactorisation.  The staged
// transform kernels are templates in qst_stages.hpp, instantiated in
// qst_lo_f32.hip, qst_lo_f64.hip and qst_hi.hip.
#include "qst_device.hpp"
#include "qst_internal.hpp"

namespace qst {

// ------------------------------------------------------------------ decode
// Settings [B][N] uint8 -> 2-bit codes packed by index bit: qubit j sits at bit
// N-1-j, so its code occupies bits 2(N-1-j) .. 2(N-1-j)+1.  Codes > 2 are
// treated as Z and raise *flag.
__global__ void k_decode(const uint8_t* __restrict__ settings, int B, int N, uint64_t* __restrict__ pc,
                         int* __restrict__ flag) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  uint64_t v = 0;
  int bad = 0;
  for (int j = 0; j < N; ++j) {
    uint32_t c = settings[(size_t)b * N + j];
    if (c > 2u) {
      bad = 1;
      c = 2u;
    }
    v |= (uint64_t)c << (2 * (N - 1 - j));
  }
  pc[b] = v;
  if (bad) atomicOr(flag, 1);
}

hipError_t launch_decode(const uint8_t* settings, int B, int N, uint64_t* pc, int* flag, hipStream_t st) {
  const int bs = 256;
  k_decode<<<(B + bs - 1) / bs, bs, 0, st>>>(settings, B, N, pc, flag);
  return hipGetLastError();
}

// General local settings: thread (b, j) writes the rotation form of qubit j of setting b
// at um[(b N + N-1-j) 8 ..]: the matrix U (the Pauli rotations for codes 0..2, V_Z = I,
// unitaries[code - 3] beyond) is P R diag(1, e) with P diagonal unitary, R = [[c, -s], [s, c]],
// c = |u00|, s = |u10| and e = c u11' - s u01' (u' = the second column with P's phases
// removed).  P multiplies each outcome's amplitude by a phase, which changes neither |phi|^2
// nor V^dagger diag(g) V, so only (tan(theta/2) = s / (1 + c), s, Re e, Im e) are stored
// (FP32, computed in FP64; theta in [0, pi/2] since c, s >= 0).
// A table entry that is not unitary to 1e-6 ORs 2 into the flag and acts as the identity;
// codes beyond the table OR in 1 (identity).  pc gets code 0 everywhere.
__global__ void k_decode_general(const uint8_t* __restrict__ settings, int B, int N,
                                 const double* __restrict__ unitaries, int K, float* __restrict__ um,
                                 uint64_t* __restrict__ pc, int* __restrict__ flag) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= (long long)B * N) return;
  const int b = (int)(t / N);
  const int j = (int)(t - (long long)b * N);
  const uint32_t c = settings[t];
  constexpr double r2 = 0.70710678118654752440;
  // u00, u01, u10, u11 as (re, im)
  double u[8] = {1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0};
  if (c == 0u) {
    const double v[8] = {r2, 0.0, r2, 0.0, r2, 0.0, -r2, 0.0};
    for (int k = 0; k < 8; ++k) u[k] = v[k];
  } else if (c == 1u) {
    const double v[8] = {r2, 0.0, 0.0, -r2, r2, 0.0, 0.0, r2};
    for (int k = 0; k < 8; ++k) u[k] = v[k];
  } else if (c >= 3u) {
    if ((int)(c - 3u) < K) {
      const double* m = unitaries + (size_t)(c - 3u) * 8;
      for (int k = 0; k < 8; ++k) u[k] = m[k];
      // U^dagger U = I: unit columns, orthogonal to each other
      const double n0 = u[0] * u[0] + u[1] * u[1] + u[4] * u[4] + u[5] * u[5];
      const double n1 = u[2] * u[2] + u[3] * u[3] + u[6] * u[6] + u[7] * u[7];
      const double ore = u[0] * u[2] + u[1] * u[3] + u[4] * u[6] + u[5] * u[7];
      const double oim = u[0] * u[3] - u[1] * u[2] + u[4] * u[7] - u[5] * u[6];
      const bool ok = fabs(n0 - 1.0) <= 1e-6 && fabs(n1 - 1.0) <= 1e-6 && fabs(ore) <= 1e-6 && fabs(oim) <= 1e-6;
      if (!ok) {
        atomicOr(flag, 2);
        const double id[8] = {1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0};
        for (int k = 0; k < 8; ++k) u[k] = id[k];
      }
    } else {
      atomicOr(flag, 1);
    }
  }
  const double ca = hypot(u[0], u[1]), sa = hypot(u[4], u[5]);
  // phases conj(u00)/|u00| and conj(u10)/|u10| (1 for a zero entry)
  const double p0r = ca > 0.0 ? u[0] / ca : 1.0, p0i = ca > 0.0 ? -u[1] / ca : 0.0;
  const double p1r = sa > 0.0 ? u[4] / sa : 1.0, p1i = sa > 0.0 ? -u[5] / sa : 0.0;
  const double br = p0r * u[2] - p0i * u[3], bi = p0r * u[3] + p0i * u[2];  // u01'
  const double dr = p1r * u[6] - p1i * u[7], di = p1r * u[7] + p1i * u[6];  // u11'
  const double er = ca * dr - sa * br, ei = ca * di - sa * bi;
  float* dst = um + ((size_t)b * N + (N - 1 - j)) * 8;
  dst[0] = (float)(sa / (1.0 + ca));
  dst[1] = (float)sa;
  dst[2] = (float)er;
  dst[3] = (float)ei;
  for (int k = 4; k < 8; ++k) dst[k] = 0.f;
  if (j == 0) pc[b] = 0ull;
}

hipError_t launch_decode_general(const uint8_t* settings, int B, int N, const double* unitaries, int K, float* um,
                                 uint64_t* pc, int* flag, hipStream_t st) {
  const long long n = (long long)B * N;
  const int bs = 256;
  k_decode_general<<<(unsigned)((n + bs - 1) / bs), bs, 0, st>>>(settings, B, N, unitaries, K, um, pc, flag);
  return hipGetLastError();
}

// ------------------------------------------------------------------ sparse frequencies
__device__ __forceinline__ long long clamp_ll(long long v, long long lo, long long hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

// First position in [lo, hi) whose outcome is >= target (idx ascending within a row).
__device__ __forceinline__ long long lower_bound_idx(const int* __restrict__ idx, long long lo, long long hi,
                                                     long long target) {
  while (lo < hi) {
    const long long mid = lo + ((hi - lo) >> 1);
    if ((long long)idx[mid] < target)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

__global__ void k_chunk_ptr(const long long* __restrict__ rowptr, const int* __restrict__ idx, long long nnz, int B,
                            int nh, int U, long long* __restrict__ cptr) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const long long n = (long long)B * nh;
  if (t > n) return;
  if (t == n) {
    cptr[n] = nnz;
    return;
  }
  const int b = (int)(t / nh);
  const int hh = (int)(t - (long long)b * nh);
  const long long lo = clamp_ll(rowptr[b], 0, nnz);
  const long long hi = clamp_ll(rowptr[b + 1], lo, nnz);
  cptr[t] = lower_bound_idx(idx, lo, hi, (long long)hh * U);
}

hipError_t launch_chunk_ptr(const long long* rowptr, const int* idx, long long nnz, int B, int nh, int U,
                            long long* cptr, hipStream_t st) {
  const long long n = (long long)B * nh + 1;
  const int bs = 256;
  k_chunk_ptr<<<(unsigned)((n + bs - 1) / bs), bs, 0, st>>>(rowptr, idx, nnz, B, nh, U, cptr);
  return hipGetLastError();
}

// ------------------------------------------------------------------ fill
__global__ void k_fill(uint32_t* p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0u;
}

hipError_t launch_fill(void* p, size_t bytes, hipStream_t st) {
  const size_t n = bytes / 4;
  if (n == 0) return hipSuccess;
  const int bs = 256;
  const size_t g = (n + bs - 1) / bs;
  k_fill<<<(unsigned)(g < 4096 ? g : 4096), bs, 0, st>>>(reinterpret_cast<uint32_t*>(p), n);
  return hipGetLastError();
}

// ------------------------------------------------------------------ stage B
// Low-stage LDS: the transpose planes, the |phi|^2 table [R][Upad] and the
// sensitivity row [Upad] (layouts below), then one double per thread for the
// reductions.
size_t lo_lds_bytes_logv(const Geometry& g, int logv) {
  const size_t U = (size_t)1 << g.n_lo;
  const size_t Upad = U + (U >> 5);
  const size_t nthr = (size_t)g.R << (g.n_lo - logv);
  // Wavefront-local transposes (at most 64 threads per atom): one plane per atom
  // plus a separate |phi|^2 table and g row; otherwise two planes per atom that
  // the table and the g row alias.
  const bool wave_local = g.n_lo - logv <= 6;
  const size_t rows = wave_local ? 2 * (size_t)g.R + 1 : 2 * (size_t)g.R;
  const size_t planes = ((rows * Upad * g.elem) + 15) & ~(size_t)15;
  return planes + nthr * sizeof(double);
}

size_t lo_lds_bytes(const Geometry& g) {
  const bool staged = g.n_hi > 0;
  const size_t f = lo_lds_bytes_logv(g, lo_logv_of(g.n_lo, staged, false));
  const size_t b = lo_lds_bytes_logv(g, lo_logv_of(g.n_lo, staged, true));
  return f > b ? f : b;
}

// ------------------------------------------------------------------ stage dispatch
hipError_t launch_stage_lo_f32(const Geometry& g, const LoBatch& m, bool adjoint, hipStream_t st);
hipError_t launch_stage_lo_h16(const Geometry& g, const LoBatch& m, bool adjoint, hipStream_t st);
hipError_t launch_stage_lo_f64(const Geometry& g, const LoBatch& m, bool adjoint, hipStream_t st);
hipError_t launch_stage_lo_gen(const Geometry& g, const LoBatch& m, bool adjoint, hipStream_t st);
int lo_occupancy_f32(const Geometry& g);
int lo_occupancy_gen(const Geometry& g);
int lo_occupancy_h16(const Geometry& g);
int lo_occupancy_f64(const Geometry& g);

hipError_t launch_stage_lo(const Geometry& g, const LoBatch& m, bool adjoint, hipStream_t st) {
  if (m.count < 1 || m.count > kBatchMax || m.rmax != g.R) return hipErrorInvalidValue;
  if (g.elem != 4) return g.gen ? hipErrorInvalidValue : launch_stage_lo_f64(g, m, adjoint, st);
  if (g.gen) return g.h16 ? hipErrorInvalidValue : launch_stage_lo_gen(g, m, adjoint, st);
  return g.h16 ? launch_stage_lo_h16(g, m, adjoint, st) : launch_stage_lo_f32(g, m, adjoint, st);
}

// Resident low-stage work-groups per compute unit (the persistent grid is this
// times the number of compute units).
int lo_blocks_per_cu(const Geometry& g) {
  if (g.elem != 4) return lo_occupancy_f64(g);
  if (g.gen) return lo_occupancy_gen(g);
  return g.h16 ? lo_occupancy_h16(g) : lo_occupancy_f32(g);
}

size_t hi_lds_bytes(const Geometry& g) {
  const size_t N = (size_t)1 << g.t;
  return (N + (N >> 5)) * 2 * (size_t)g.elem;
}

// ------------------------------------------------------------------ sum over settings (no high bits)
// grad[e] (+)= sum_s W[s][e].  A block takes kSumCols consecutive elements; for each,
// kSumSlices threads sum the settings s = slice, slice + kSumSlices, ... in increasing
// order, and the slice sums are added in a fixed tree.  The single-instance and the
// batched kernels share this order, so both give the same bits.
constexpr int kSumSlices = 8;
constexpr int kSumCols = 32;

template <typename T, bool H16>
__device__ __forceinline__ cx<T> w_at(const void* W, long long i) {
  if constexpr (H16) {
    const uint32_t w = reinterpret_cast<const uint32_t*>(W)[i];
    return cx<T>{__uint_as_float(w << 16), __uint_as_float(w & 0xffff0000u)};
  } else {
    return reinterpret_cast<const cx<T>*>(W)[i];
  }
}

template <typename T, bool H16>
__device__ __forceinline__ cx<T> settings_slice(const void* __restrict__ W, int S, long long RD, long long e, int sl) {
  cx<T> a{0, 0};
  for (int s = sl; s < S; s += kSumSlices) {
    const cx<T> w = w_at<T, H16>(W, (long long)s * RD + e);
    a.x += w.x;
    a.y += w.y;
  }
  return a;
}

template <typename T>
__device__ __forceinline__ cx<T> slice_tree(const cx<T> (*part)[kSumCols], int col) {
  auto add = [](cx<T> a, cx<T> b) { return cx<T>{a.x + b.x, a.y + b.y}; };
  const cx<T> p01 = add(part[0][col], part[1][col]), p23 = add(part[2][col], part[3][col]);
  const cx<T> p45 = add(part[4][col], part[5][col]), p67 = add(part[6][col], part[7][col]);
  return add(add(p01, p23), add(p45, p67));
}

template <typename T, bool H16>
__global__ __launch_bounds__(kSumSlices * kSumCols) void k_sum_settings(const void* __restrict__ W, int S, long long RD,
                                                                        cx<T>* __restrict__ grad, int first) {
  __shared__ cx<T> part[kSumSlices][kSumCols];
  const int col = threadIdx.x % kSumCols, sl = threadIdx.x / kSumCols;
  for (long long e0 = blockIdx.x * (long long)kSumCols; e0 < RD; e0 += (long long)gridDim.x * kSumCols) {
    const long long e = e0 + col;
    part[sl][col] = e < RD ? settings_slice<T, H16>(W, S, RD, e, sl) : cx<T>{0, 0};
    __syncthreads();
    if (sl == 0 && e < RD) {
      const cx<T> acc = slice_tree<T>(part, col);
      if (first) {
        grad[e] = acc;
      } else {
        const cx<T> x = grad[e];
        grad[e] = cx<T>{x.x + acc.x, x.y + acc.y};
      }
    }
    __syncthreads();
  }
}

hipError_t launch_sum_settings(const Geometry& g, const void* W, int S, void* grad, int first, hipStream_t st) {
  const long long RD = (long long)g.R * g.D;
  long long nb = (RD + kSumCols - 1) / kSumCols;
  if (nb > 8192) nb = 8192;
  const int bs = kSumSlices * kSumCols;
  if (g.elem == 4 && g.h16)
    k_sum_settings<float, true><<<(unsigned)nb, bs, 0, st>>>(W, S, RD, reinterpret_cast<float2*>(grad), first);
  else if (g.elem == 4)
    k_sum_settings<float, false><<<(unsigned)nb, bs, 0, st>>>(W, S, RD, reinterpret_cast<float2*>(grad), first);
  else
    k_sum_settings<double, false><<<(unsigned)nb, bs, 0, st>>>(W, S, RD, reinterpret_cast<double2*>(grad), first);
  return hipGetLastError();
}

template <typename T>
__global__ void k_sum_splits(const cx<T>* __restrict__ part, int nsplit, long long RD, cx<T>* __restrict__ grad,
                             int first) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < RD; e += (long long)gridDim.x * blockDim.x) {
    cx<T> acc = first ? cx<T>{0, 0} : grad[e];
    for (int k = 0; k < nsplit; ++k) {
      const cx<T> v = part[(long long)k * RD + e];
      acc.x += v.x;
      acc.y += v.y;
    }
    grad[e] = acc;
  }
}

hipError_t launch_sum_splits(int elem, const void* part, int nsplit, long long RD, void* grad, int first,
                             hipStream_t st) {
  const int bs = 256;
  long long nb = (RD + bs - 1) / bs;
  if (nb > 8192) nb = 8192;
  if (elem == 4)
    k_sum_splits<float><<<(unsigned)nb, bs, 0, st>>>(reinterpret_cast<const float2*>(part), nsplit, RD,
                                                      reinterpret_cast<float2*>(grad), first);
  else
    k_sum_splits<double><<<(unsigned)nb, bs, 0, st>>>(reinterpret_cast<const double2*>(part), nsplit, RD,
                                                       reinterpret_cast<double2*>(grad), first);
  return hipGetLastError();
}

hipError_t launch_plain_sum(const void* X, int S, int R, long long D, void* grad, int first, hipStream_t st) {
  Geometry g{};
  g.R = R;
  g.D = D;
  g.elem = 4;
  return launch_sum_settings(g, X, S, grad, first, st);
}

// ------------------------------------------------------------------ deterministic reductions
__device__ __forceinline__ double block_tree(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int st = blockDim.x >> 1; st > 0; st >>= 1) {
    if (tid < st) red[tid] += red[tid + st];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// part [rows][nslots] -> lvl1 [rows][g1]; block b sums a contiguous range of slots.
__global__ __launch_bounds__(256) void k_rowsum1(const double* __restrict__ part, long long nslots, double* lvl1,
                                                 int g1) {
  __shared__ double red[256];
  const int row = blockIdx.y, blk = blockIdx.x;
  const long long per = (nslots + g1 - 1) / g1;
  const long long beg = (long long)blk * per;
  long long end = beg + per;
  if (end > nslots) end = nslots;
  double acc = 0.0;
  for (long long i = beg + threadIdx.x; i < end; i += 256) acc += part[(long long)row * nslots + i];
  const double r = block_tree(acc, red);
  if (threadIdx.x == 0) lvl1[(long long)row * g1 + blk] = r;
}

__global__ __launch_bounds__(256) void k_rowsum2(const double* __restrict__ lvl1, int g1, double* out) {
  __shared__ double red[256];
  const int row = blockIdx.x;
  double acc = 0.0;
  for (int i = threadIdx.x; i < g1; i += 256) acc += lvl1[(long long)row * g1 + i];
  const double r = block_tree(acc, red);
  if (threadIdx.x == 0) out[row] = r;
}

hipError_t launch_rowsum(const double* part, int rows, long long nslots, double* lvl1, int g1, double* out,
                         hipStream_t st) {
  k_rowsum1<<<dim3(g1, rows), 256, 0, st>>>(part, nslots, lvl1, g1);
  k_rowsum2<<<rows, 256, 0, st>>>(lvl1, g1, out);
  return hipGetLastError();
}

__global__ void k_scatter(const double* sums, int R, double* loss, double* wgrad) {
  const int i = threadIdx.x;
  if (i == 0 && loss) *loss = sums[0];
  if (wgrad && i < R) wgrad[i] = sums[1 + i];
}

hipError_t launch_scatter_results(const double* sums, int R, double* loss, double* wgrad, hipStream_t st) {
  k_scatter<<<1, (R + 1 + 63) / 64 * 64, 0, st>>>(sums, R, loss, wgrad);
  return hipGetLastError();
}

// ------------------------------------------------------------------ tangent projection (optional epilogue)
template <typename T>
__global__ __launch_bounds__(256) void k_tan_dot(const cx<T>* __restrict__ psi, const cx<T>* __restrict__ grad,
                                                 long long D, double* part, int g1) {
  __shared__ double red[256];
  const int r = blockIdx.y, blk = blockIdx.x;
  const long long per = (D + g1 - 1) / g1;
  const long long beg = (long long)blk * per;
  long long end = beg + per;
  if (end > D) end = D;
  double re = 0.0, im = 0.0;
  for (long long i = beg + threadIdx.x; i < end; i += 256) {
    const cx<T> p = psi[(long long)r * D + i], g = grad[(long long)r * D + i];
    re += (double)p.x * g.x + (double)p.y * g.y;  // conj(p) g
    im += (double)p.x * g.y - (double)p.y * g.x;
  }
  const double sre = block_tree(re, red);
  const double sim = block_tree(im, red);
  if (threadIdx.x == 0) {
    part[((long long)r * g1 + blk) * 2 + 0] = sre;
    part[((long long)r * g1 + blk) * 2 + 1] = sim;
  }
}

__global__ __launch_bounds__(256) void k_tan_fin(const double* part, int g1, double* dots) {
  __shared__ double red[256];
  const int r = blockIdx.x;
  double re = 0.0, im = 0.0;
  for (int i = threadIdx.x; i < g1; i += 256) {
    re += part[((long long)r * g1 + i) * 2 + 0];
    im += part[((long long)r * g1 + i) * 2 + 1];
  }
  const double sre = block_tree(re, red);
  const double sim = block_tree(im, red);
  if (threadIdx.x == 0) {
    dots[2 * r] = sre;
    dots[2 * r + 1] = sim;
  }
}

template <typename T>
__global__ void k_tan_apply(const cx<T>* __restrict__ psi, cx<T>* __restrict__ grad, int R, long long D,
                            const double* dots) {
  const long long n = (long long)R * D;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(e / D);
    const T dr = (T)dots[2 * r], di = (T)dots[2 * r + 1];
    const cx<T> p = psi[e];
    cx<T> g = grad[e];
    g.x -= p.x * dr - p.y * di;
    g.y -= p.x * di + p.y * dr;
    grad[e] = g;
  }
}

hipError_t launch_tangent(int elem, const void* atoms, void* grad, int R, long long D, double* scratch, int g1,
                          hipStream_t st) {
  double* part = scratch;
  double* dots = scratch + (size_t)R * g1 * 2;
  long long nb = ((long long)R * D + 255) / 256;
  if (nb > 8192) nb = 8192;
  if (elem == 4) {
    k_tan_dot<float><<<dim3(g1, R), 256, 0, st>>>(reinterpret_cast<const float2*>(atoms),
                                                   reinterpret_cast<const float2*>(grad), D, part, g1);
    k_tan_fin<<<R, 256, 0, st>>>(part, g1, dots);
    k_tan_apply<float><<<(unsigned)nb, 256, 0, st>>>(reinterpret_cast<const float2*>(atoms),
                                                     reinterpret_cast<float2*>(grad), R, D, dots);
  } else {
    k_tan_dot<double><<<dim3(g1, R), 256, 0, st>>>(reinterpret_cast<const double2*>(atoms),
                                                    reinterpret_cast<const double2*>(grad), D, part, g1);
    k_tan_fin<<<R, 256, 0, st>>>(part, g1, dots);
    k_tan_apply<double><<<(unsigned)nb, 256, 0, st>>>(reinterpret_cast<const double2*>(atoms),
                                                      reinterpret_cast<double2*>(grad), R, D, dots);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ batches of small instances
// Linear search for the instance of a global item index (count <= kBatchMax, uniform).
template <typename I>
__device__ __forceinline__ int batch_find(const I* begin, int count, I x) {
  int k = 0;
  while (k + 1 < count && x >= begin[k + 1]) ++k;
  return k;
}

__global__ void k_decode_batch(const DecodeBatch b, int* __restrict__ flag) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= b.total) return;
  const int k = batch_find(b.begin, b.count, t);
  const int row = t - b.begin[k];
  uint64_t v = 0;
  int bad = 0;
  for (int j = 0; j < b.N; ++j) {
    uint32_t c = b.settings[k][(size_t)row * b.N + j];
    if (c > 2u) {
      bad = 1;
      c = 2u;
    }
    v |= (uint64_t)c << (2 * (b.N - 1 - j));
  }
  b.pc[k][row] = v;
  if (bad) atomicOr(flag, 1);
}

hipError_t launch_decode_batch(const DecodeBatch& b, int* flag, hipStream_t st) {
  if (b.total < 1) return hipSuccess;
  const int bs = 256;
  k_decode_batch<<<(b.total + bs - 1) / bs, bs, 0, st>>>(b, flag);
  return hipGetLastError();
}

template <typename T, bool H16>
__global__ __launch_bounds__(kSumSlices * kSumCols) void k_sum_batch(const SumBatch b) {
  __shared__ cx<T> part[kSumSlices][kSumCols];
  const int col = threadIdx.x % kSumCols, sl = threadIdx.x / kSumCols;
  for (long long t0 = blockIdx.x * (long long)kSumCols; t0 < b.total; t0 += (long long)gridDim.x * kSumCols) {
    const long long t = t0 + col;
    int k = 0;
    long long e = 0;
    if (t < b.total) {
      k = batch_find(b.begin, b.count, t);
      e = t - b.begin[k];
      part[sl][col] = settings_slice<T, H16>(b.W[k], b.S[k], b.RD[k], e, sl);
    } else {
      part[sl][col] = cx<T>{0, 0};
    }
    __syncthreads();
    if (sl == 0 && t < b.total) reinterpret_cast<cx<T>*>(b.grad[k])[e] = slice_tree<T>(part, col);
    __syncthreads();
  }
}

hipError_t launch_sum_batch(const SumBatch& b, hipStream_t st) {
  if (b.total < 1) return hipSuccess;
  long long nb = (b.total + kSumCols - 1) / kSumCols;
  if (nb > 8192) nb = 8192;
  const int bs = kSumSlices * kSumCols;
  if (b.elem == 4 && b.h16)
    k_sum_batch<float, true><<<(unsigned)nb, bs, 0, st>>>(b);
  else if (b.elem == 4)
    k_sum_batch<float, false><<<(unsigned)nb, bs, 0, st>>>(b);
  else
    k_sum_batch<double, false><<<(unsigned)nb, bs, 0, st>>>(b);
  return hipGetLastError();
}

// Work-group (k, row): row 0 is instance k's loss, rows 1..R_k its weight gradient.
__global__ __launch_bounds__(256) void k_rowsum_batch(const RowBatch b) {
  __shared__ double red[256];
  const int k = blockIdx.x, row = blockIdx.y;
  if (row > b.R[k]) return;
  if (row == 0 && b.loss[k] == nullptr) return;
  if (row > 0 && b.wgrad[k] == nullptr) return;
  double acc = 0.0;
  for (long long i = threadIdx.x; i < b.nslots; i += 256) acc += b.part[k][(long long)row * b.nslots + i];
  const double r = block_tree(acc, red);
  if (threadIdx.x == 0) {
    if (row == 0)
      *b.loss[k] = r;
    else
      b.wgrad[k][row - 1] = r;
  }
}

hipError_t launch_rowsum_batch(const RowBatch& b, hipStream_t st) {
  if (b.count < 1) return hipSuccess;
  k_rowsum_batch<<<dim3(b.count, b.rmax + 1), 256, 0, st>>>(b);
  return hipGetLastError();
}

// Work-group (k, r): the FP64 inner product <psi, grad> over D, then the projection.
template <typename T>
__global__ __launch_bounds__(256) void k_tan_batch(const TanBatch b) {
  __shared__ double red[256];
  const int k = blockIdx.x, r = blockIdx.y;
  if (r >= b.R[k]) return;
  const long long D = b.D[k];
  const cx<T>* psi = reinterpret_cast<const cx<T>*>(b.atoms[k]) + (long long)r * D;
  cx<T>* grad = reinterpret_cast<cx<T>*>(b.grad[k]) + (long long)r * D;
  double re = 0.0, im = 0.0;
  for (long long i = threadIdx.x; i < D; i += 256) {
    const cx<T> p = psi[i], g = grad[i];
    re += (double)p.x * g.x + (double)p.y * g.y;  // conj(p) g
    im += (double)p.x * g.y - (double)p.y * g.x;
  }
  const T dr = (T)block_tree(re, red);
  const T di = (T)block_tree(im, red);
  for (long long i = threadIdx.x; i < D; i += 256) {
    const cx<T> p = psi[i];
    cx<T> g = grad[i];
    g.x -= p.x * dr - p.y * di;
    g.y -= p.x * di + p.y * dr;
    grad[i] = g;
  }
}

hipError_t launch_tangent_batch(const TanBatch& b, hipStream_t st) {
  if (b.count < 1) return hipSuccess;
  if (b.elem == 4)
    k_tan_batch<float><<<dim3(b.count, b.rmax), 256, 0, st>>>(b);
  else
    k_tan_batch<double><<<dim3(b.count, b.rmax), 256, 0, st>>>(b);
  return hipGetLastError();
}

// ------------------------------------------------------------------ simplex reweight (FP64, one work-group)
// beta = proj_simplex(alpha + eta h) by the sort-free rank form of the sort-based
// projection: element i sits at sorted position k_i (ties by index); the support
// size is the largest k_i with v_i - (S_i - 1)/k_i > 0, where S_i sums the k_i
// largest entries; theta = (S - 1)/k at that position.
__global__ __launch_bounds__(1024) void k_reweight(const double* __restrict__ alpha, const double* __restrict__ h,
                                                   int R, double eta, double tau, double* __restrict__ out,
                                                   int32_t* __restrict__ keep, int32_t* __restrict__ R_out) {
  __shared__ double v[1024];
  __shared__ double beta[1024];
  __shared__ int kk[1024];
  __shared__ double theta_s;
  __shared__ double sum_s;
  __shared__ int rho_s, cnt_s, arg_s;
  const int i = threadIdx.x;
  if (i < R) v[i] = alpha[i] + eta * h[i];
  __syncthreads();
  int k = 0;
  double S = 0.0;
  if (i < R) {
    k = 1;
    S = v[i];
    for (int j = 0; j < R; ++j) {
      if (j == i) continue;
      if (v[j] > v[i] || (v[j] == v[i] && j < i)) {
        ++k;
        S += v[j];
      }
    }
    kk[i] = (v[i] - (S - 1.0) / k > 0.0) ? k : 0;
  }
  __syncthreads();
  if (i == 0) {
    int rho = 0;
    for (int j = 0; j < R; ++j) rho = kk[j] > rho ? kk[j] : rho;
    rho_s = rho;
  }
  __syncthreads();
  if (i < R && k == rho_s) theta_s = (S - 1.0) / k;
  __syncthreads();
  if (i < R) beta[i] = fmax(v[i] - theta_s, 0.0);
  __syncthreads();
  if (i == 0) {
    int cnt = 0, arg = 0;
    double sum = 0.0, best = -1.0;
    for (int j = 0; j < R; ++j) {
      if (beta[j] > tau) {
        ++cnt;
        sum += beta[j];
      }
      if (beta[j] > best) {
        best = beta[j];
        arg = j;
      }
    }
    const int fallback = cnt == 0;  // nothing above tau: keep the first maximum alone
    if (fallback) {
      cnt = 1;
      sum = beta[arg];
    }
    cnt_s = cnt;
    sum_s = sum;
    arg_s = fallback ? arg : -1;
    *R_out = cnt;
  }
  __syncthreads();
  if (i < R) {
    const bool fallback = arg_s >= 0;
    const bool kept = fallback ? (i == arg_s) : (beta[i] > tau);
    if (kept) {
      int slot = 0;
      if (!fallback)
        for (int j = 0; j < i; ++j) slot += beta[j] > tau ? 1 : 0;
      out[slot] = beta[i] / sum_s;
      keep[slot] = i;
    }
    if (i >= cnt_s) {
      out[i] = 0.0;
      keep[i] = -1;
    }
  }
}

hipError_t launch_reweight(const double* alpha, const double* h, int R, double eta, double tau, double* alpha_out,
                           int32_t* keep, int32_t* R_out, hipStream_t st) {
  const int bs = (R + 63) / 64 * 64;
  k_reweight<<<1, bs, 0, st>>>(alpha, h, R, eta, tau, alpha_out, keep, R_out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ atom-step pair (eq. pi-update)
// pair[0] = psi_trial, pair[1] = atoms[r]; wpair = (alpha_r, -alpha_r).  Elements are
// copied as 8-byte words (elem_words per complex: 1 for complex64, 2 for complex128).
__global__ void k_atom_pair(const unsigned long long* __restrict__ trial, const unsigned long long* __restrict__ atoms,
                            const double* __restrict__ alpha, int r, long long words,
                            unsigned long long* __restrict__ pair, double* __restrict__ wpair) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < words; e += stride) {
    pair[e] = trial[e];
    pair[words + e] = atoms[(long long)r * words + e];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    wpair[0] = alpha[r];
    wpair[1] = -alpha[r];
  }
}

hipError_t launch_atom_pair(int elem, const void* trial, const void* atoms, const double* alpha, int r, long long D,
                            void* pair, double* wpair, hipStream_t st) {
  const long long words = D * (elem == 8 ? 2 : 1);
  long long nb = (words + 255) / 256;
  if (nb > 8192) nb = 8192;
  k_atom_pair<<<(unsigned)nb, 256, 0, st>>>(reinterpret_cast<const unsigned long long*>(trial),
                                           reinterpret_cast<const unsigned long long*>(atoms), alpha, r, words,
                                           reinterpret_cast<unsigned long long*>(pair), wpair);
  return hipGetLastError();
}

// ------------------------------------------------------------------ plain per-qubit reference path (FP32)
__global__ void k_plain_copy(const float2* __restrict__ psi, float2* __restrict__ X, int S, long long RD) {
  const long long n = (long long)S * RD;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
    X[e] = psi[e % RD];
}

hipError_t launch_plain_copy(const void* atoms, void* X, int S, int R, long long D, hipStream_t st) {
  const long long RD = (long long)R * D;
  long long nb = ((long long)S * RD + 255) / 256;
  if (nb > 65536) nb = 65536;
  k_plain_copy<<<(unsigned)nb, 256, 0, st>>>(reinterpret_cast<const float2*>(atoms), reinterpret_cast<float2*>(X), S,
                                            RD);
  return hipGetLastError();
}

// One butterfly pass over index bit `bit` for every (setting, atom) vector of X.
template <bool ADJ>
__global__ void k_plain_qubit(float2* __restrict__ X, int S, int R, long long D, int bit,
                              const uint64_t* __restrict__ pc, int b0) {
  const long long half = D >> 1;
  const long long per_set = (long long)R * half;
  const long long n = (long long)S * per_set;
  const long long lowmask = (1ll << bit) - 1;
  for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
    const int s = (int)(q / per_set);
    const uint32_t code = (uint32_t)((pc[b0 + s] >> (2 * bit)) & 3ull);
    if (code >= 2u) continue;
    const long long rem = q - (long long)s * per_set;
    const long long vec = (long long)s * R + rem / half;
    const long long p = rem % half;
    const long long i0 = ((p & ~lowmask) << 1) | (p & lowmask);
    float2* base = X + vec * D;
    float2 a = base[i0], b = base[i0 | (1ll << bit)];
    if (code == 0u)
      bf_x(a, b);
    else if (ADJ)
      bf_yh(a, b);
    else
      bf_y(a, b);
    base[i0] = a;
    base[i0 | (1ll << bit)] = b;
  }
}

hipError_t launch_plain_qubit(void* X, int S, int R, long long D, int bit, const uint64_t* pc, int b0, bool adj,
                              hipStream_t st) {
  const long long n = (long long)S * R * (D >> 1);
  long long nb = (n + 255) / 256;
  if (nb > 65536) nb = 65536;
  if (adj)
    k_plain_qubit<true><<<(unsigned)nb, 256, 0, st>>>(reinterpret_cast<float2*>(X), S, R, D, bit, pc, b0);
  else
    k_plain_qubit<false><<<(unsigned)nb, 256, 0, st>>>(reinterpret_cast<float2*>(X), S, R, D, bit, pc, b0);
  return hipGetLastError();
}

// Pointwise step of the plain path: one thread per (setting, outcome), all atoms.
// Slots: one per (setting, block of 256 outcomes).
__global__ __launch_bounds__(256) void k_plain_point(const LoArgs a, float2* __restrict__ X, int S) {
  __shared__ double red[256];
  const long long D = a.D;
  const long long nblk = (D + 255) / 256;
  const int s = (int)(blockIdx.x / nblk);
  const long long blk = blockIdx.x - (long long)s * nblk;
  const int b = a.b0 + s;
  const uint64_t pc = a.pc[b];
  const float s2 = (float)ldexp(1.0, -nonz_count(pc, a.n));
  const long long u = blk * 256 + threadIdx.x;
  const double Bd = (double)a.B;
  const bool in = u < D;
  double loss = 0.0;
  float g = 0.0f;
  if (in) {
    float p = 0.0f;
    for (int r = 0; r < a.R; ++r) {
      const float2 x = X[((long long)s * a.R + r) * D + u];
      p += (float)a.alpha[r] * (x.x * x.x + x.y * x.y);
    }
    p *= s2;
    const long long gi = (long long)b * D + u;
    if (a.pbase) p += reinterpret_cast<const float*>(a.pbase)[gi];
    if (a.probs) reinterpret_cast<float*>(a.probs)[gi] = p;
    if (a.grad_p) {
      g = reinterpret_cast<const float*>(a.grad_p)[gi];
    } else if (a.loss_kind == 0) {
      double f = 0.0;
      if (a.fidx) {  // sparse: row b's non-zeros are [fchunk[b], fchunk[b + 1])
        const long long e0 = a.fchunk[b], e1 = a.fchunk[b + 1] > e0 ? a.fchunk[b + 1] : e0;
        const long long e = lower_bound_idx(a.fidx, e0, e1, u);
        if (e < e1 && (long long)a.fidx[e] == u) f = (double)a.freqs[e];
      } else {
        f = (double)a.freqs[gi];
      }
      if (f > 0.0) {
        const double piv = (double)p / Bd + a.eps;
        loss = -(f / Bd) * log(piv);
        g = (float)(-(f / Bd) / piv / Bd);
      }
    } else if (a.loss_kind == 1) {
      double f = 0.0;
      if (a.fidx) {
        const long long e0 = a.fchunk[b], e1 = a.fchunk[b + 1] > e0 ? a.fchunk[b + 1] : e0;
        const long long e = lower_bound_idx(a.fidx, e0, e1, u);
        if (e < e1 && (long long)a.fidx[e] == u) f = (double)a.freqs[e];
      } else {
        f = (double)a.freqs[gi];
      }
      const double rr = ((double)p - f) / Bd;
      loss = 0.5 * rr * rr;
      g = (float)(rr / Bd);
    }
  }
  const long long slot = (long long)b * nblk + blk;
  const float gs = g * s2;
  for (int r = 0; r < a.R; ++r) {
    double hr = 0.0;
    if (in) {
      float2* xp = X + ((long long)s * a.R + r) * D + u;
      const float2 x = *xp;
      hr = (double)(gs * (x.x * x.x + x.y * x.y));
      const float sc = (float)a.alpha[r] * gs;
      *xp = float2{x.x * sc, x.y * sc};
    }
    if (a.part) {
      const double t = block_tree(hr, red);
      if (threadIdx.x == 0) a.part[(long long)(1 + r) * a.nslots + slot] = t;
    }
  }
  if (a.part && a.grad_p == nullptr && a.loss_kind != 2) {
    const double t = block_tree(loss, red);
    if (threadIdx.x == 0) a.part[slot] = t;
  }
}

hipError_t launch_plain_point(const LoArgs& a, void* X, int S, hipStream_t st) {
  const long long nblk = (a.D + 255) / 256;
  k_plain_point<<<(unsigned)(S * nblk), 256, 0, st>>>(a, reinterpret_cast<float2*>(X), S);
  return hipGetLastError();
}

// ------------------------------------------------------------------ vector helpers (refactorisation)
template <typename CW>
__device__ __forceinline__ double2 ld_c(const CW* p, long long i);
template <>
__device__ __forceinline__ double2 ld_c<double2>(const double2* p, long long i) {
  return p[i];
}
template <>
__device__ __forceinline__ double2 ld_c<float2>(const float2* p, long long i) {
  const float2 x = p[i];
  return double2{(double)x.x, (double)x.y};
}

// out[j] = <q_j, w> = sum conj(q_j) w  for j < k.   Q [k][ldq] complex128.
template <typename CW>
__global__ __launch_bounds__(256) void k_dots1(const double2* __restrict__ Q, long long ldq,
                                               const CW* __restrict__ w, long long D, double* part, int g1) {
  __shared__ double red[256];
  const int j = blockIdx.y, blk = blockIdx.x;
  const long long per = (D + g1 - 1) / g1;
  const long long beg = (long long)blk * per;
  long long end = beg + per;
  if (end > D) end = D;
  double re = 0.0, im = 0.0;
  for (long long i = beg + threadIdx.x; i < end; i += 256) {
    const double2 q = Q[(long long)j * ldq + i];
    const double2 x = ld_c<CW>(w, i);
    re += q.x * x.x + q.y * x.y;
    im += q.x * x.y - q.y * x.x;
  }
  const double sre = block_tree(re, red);
  const double sim = block_tree(im, red);
  if (threadIdx.x == 0) {
    part[((long long)j * g1 + blk) * 2] = sre;
    part[((long long)j * g1 + blk) * 2 + 1] = sim;
  }
}

hipError_t launch_dots(const void* Q, int k, long long ldq, const void* w, int w_is_c64, long long D, double* part,
                       int g1, double* out, hipStream_t st) {
  if (k <= 0) return hipSuccess;
  if (w_is_c64)
    k_dots1<float2><<<dim3(g1, k), 256, 0, st>>>(reinterpret_cast<const double2*>(Q), ldq,
                                                 reinterpret_cast<const float2*>(w), D, part, g1);
  else
    k_dots1<double2><<<dim3(g1, k), 256, 0, st>>>(reinterpret_cast<const double2*>(Q), ldq,
                                                  reinterpret_cast<const double2*>(w), D, part, g1);
  k_tan_fin<<<k, 256, 0, st>>>(part, g1, out);
  return hipGetLastError();
}

// w += sign * sum_j coef_j q_j   (w complex128 [D]; q complex128 or complex64 rows)
template <typename CQ>
__global__ void k_combine(double2* __restrict__ w, const CQ* __restrict__ Q, int k, long long ldq,
                          const double* __restrict__ coef, double sign, long long D) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < D; i += (long long)gridDim.x * blockDim.x) {
    double re = 0.0, im = 0.0;
    for (int j = 0; j < k; ++j) {
      const double2 q = ld_c<CQ>(Q + (long long)j * ldq, i);
      const double cr = coef[2 * j], ci = coef[2 * j + 1];
      re += cr * q.x - ci * q.y;
      im += cr * q.y + ci * q.x;
    }
    double2 x = w[i];
    x.x += sign * re;
    x.y += sign * im;
    w[i] = x;
  }
}

hipError_t launch_combine(void* w, const void* Q, int k, long long ldq, const double* coef, double sign, int q_is_c64,
                          long long D, hipStream_t st) {
  if (k <= 0) return hipSuccess;
  long long nb = (D + 255) / 256;
  if (nb > 8192) nb = 8192;
  if (q_is_c64)
    k_combine<float2><<<(unsigned)nb, 256, 0, st>>>(reinterpret_cast<double2*>(w), reinterpret_cast<const float2*>(Q), k,
                                                    ldq, coef, sign, D);
  else
    k_combine<double2><<<(unsigned)nb, 256, 0, st>>>(reinterpret_cast<double2*>(w), reinterpret_cast<const double2*>(Q),
                                                     k, ldq, coef, sign, D);
  return hipGetLastError();
}

__global__ void k_convert(const void* src, int src_c64, void* dst, int dst_c64, long long n, double scale) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    double2 x = src_c64 ? ld_c<float2>(reinterpret_cast<const float2*>(src), i)
                        : reinterpret_cast<const double2*>(src)[i];
    x.x *= scale;
    x.y *= scale;
    if (dst_c64)
      reinterpret_cast<float2*>(dst)[i] = float2{(float)x.x, (float)x.y};
    else
      reinterpret_cast<double2*>(dst)[i] = x;
  }
}

hipError_t launch_convert(const void* src, int src_c64, void* dst, int dst_c64, long long n, double scale,
                          hipStream_t st) {
  long long nb = (n + 255) / 256;
  if (nb > 8192) nb = 8192;
  if (nb < 1) return hipSuccess;
  k_convert<<<(unsigned)nb, 256, 0, st>>>(src, src_c64, dst, dst_c64, n, scale);
  return hipGetLastError();
}

__global__ void k_axpy_c(void* y, int y_c64, const void* x, int x_c64, long long n, double a) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double2 xv = x_c64 ? ld_c<float2>(reinterpret_cast<const float2*>(x), i)
                             : reinterpret_cast<const double2*>(x)[i];
    if (y_c64) {
      float2* yp = reinterpret_cast<float2*>(y) + i;
      *yp = float2{(float)(yp->x + a * xv.x), (float)(yp->y + a * xv.y)};
    } else {
      double2* yp = reinterpret_cast<double2*>(y) + i;
      *yp = double2{yp->x + a * xv.x, yp->y + a * xv.y};
    }
  }
}

hipError_t launch_axpy_c(void* y, int y_c64, const void* x, int x_c64, long long n, double a, hipStream_t st) {
  long long nb = (n + 255) / 256;
  if (nb > 8192) nb = 8192;
  if (nb < 1) return hipSuccess;
  k_axpy_c<<<(unsigned)nb, 256, 0, st>>>(y, y_c64, x, x_c64, n, a);
  return hipGetLastError();
}

// ------------------------------------------------------------------ iteration helpers (Algorithm 1)
// Trial atom of eq. atom-trial: y = psi + eta * d, then y / ||y||.  Pass 1 writes y and
// per-block FP64 partials of |y|^2 (fixed grid, fixed order); the partials are summed by
// the two-level row sum; pass 2 scales by 1/sqrt(sum).
template <typename C>
__global__ __launch_bounds__(256) void k_trial_axpy(const C* __restrict__ psi, const C* __restrict__ d, double eta,
                                                    C* __restrict__ y, long long D, double* __restrict__ part) {
  __shared__ double red[256];
  double acc = 0.0;
  for (long long i = blockIdx.x * 256ll + threadIdx.x; i < D; i += (long long)gridDim.x * 256) {
    const double2 a = ld_c<C>(psi, i);
    const double2 b = ld_c<C>(d, i);
    C v;
    v.x = (decltype(v.x))fma(eta, b.x, a.x);
    v.y = (decltype(v.y))fma(eta, b.y, a.y);
    y[i] = v;
    acc += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
  }
  const double r = block_tree(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

template <typename C>
__global__ void k_scale_rsqrt(C* __restrict__ y, long long D, const double* __restrict__ sumsq) {
  const double sc = 1.0 / sqrt(*sumsq);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < D; i += (long long)gridDim.x * blockDim.x) {
    C v = y[i];
    v.x = (decltype(v.x))((double)v.x * sc);
    v.y = (decltype(v.y))((double)v.y * sc);
    y[i] = v;
  }
}

hipError_t launch_trial_atom(int elem, const void* psi, const void* d, double eta, void* y, long long D,
                             double* part, double* lvl1, int g1, double* sumsq, hipStream_t st) {
  const int nb = kTrialBlocks;
  if (elem == 8)
    k_trial_axpy<double2><<<nb, 256, 0, st>>>(reinterpret_cast<const double2*>(psi),
                                             reinterpret_cast<const double2*>(d), eta,
                                             reinterpret_cast<double2*>(y), D, part);
  else
    k_trial_axpy<float2><<<nb, 256, 0, st>>>(reinterpret_cast<const float2*>(psi),
                                            reinterpret_cast<const float2*>(d), eta, reinterpret_cast<float2*>(y),
                                            D, part);
  hipError_t e = launch_rowsum(part, 1, nb, lvl1, g1, sumsq, st);
  if (e != hipSuccess) return e;
  long long sb = (D + 255) / 256;
  if (sb > 4096) sb = 4096;
  if (elem == 8)
    k_scale_rsqrt<double2><<<(unsigned)sb, 256, 0, st>>>(reinterpret_cast<double2*>(y), D, sumsq);
  else
    k_scale_rsqrt<float2><<<(unsigned)sb, 256, 0, st>>>(reinterpret_cast<float2*>(y), D, sumsq);
  return hipGetLastError();
}

// dst row i = src row idx[i] for i < *count (rows of `words` 8-byte words); rows from
// *count to rows_max are zeroed.
__global__ void k_gather_rows(const unsigned long long* __restrict__ src, const int32_t* __restrict__ idx,
                              const int32_t* __restrict__ count, int rows_max, long long words,
                              unsigned long long* __restrict__ dst) {
  const int row = blockIdx.y;
  if (row >= rows_max) return;
  const int n = *count;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < words; e += stride)
    dst[(long long)row * words + e] = row < n ? src[(long long)idx[row] * words + e] : 0ull;
}

hipError_t launch_gather_rows(int elem, const void* src, const int32_t* idx, const int32_t* count, int rows_max,
                              long long D, void* dst, hipStream_t st) {
  if (rows_max < 1) return hipSuccess;
  const long long words = D * (elem == 8 ? 2 : 1);
  long long nb = (words + 255) / 256;
  if (nb > 2048) nb = 2048;
  k_gather_rows<<<dim3((unsigned)nb, (unsigned)rows_max), 256, 0, st>>>(
      reinterpret_cast<const unsigned long long*>(src), idx, count, rows_max, words,
      reinterpret_cast<unsigned long long*>(dst));
  return hipGetLastError();
}

}  // namespace qst
