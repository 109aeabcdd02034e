// HIP kernels of the staged butterfly path (gfx950).
//
// Forward map and adjoint of the atomic Born map over Pauli settings
// (eqs. atomic-born-map, qst-loss, likelihood-ratio-vector, weight-gradient,
// atom-wirtinger-gradient).  For setting b the rotation V_b = (x)_j V_{s_bj}
// factors over index bits, so it is applied as unscaled butterflies, one per
// non-Z qubit, with the exact scale 2^(-k_b) (k_b = non-Z count) put on |phi|^2.
//
// A state of D = 2^n amplitudes is split into low bits [0, n_lo) and high bits
// [n_lo, n).  Per batch of S settings:
//   stage A  (tile, high bits)   X[s][r] = V_b,high psi_r        (psi tile reused for S settings)
//   stage B  (chunk, low bits)   phi = V_b,low X;  p = 2^-k sum_r alpha_r |phi_r|^2;
//                                loss, g = dL/dp;  weight-gradient partials;
//                                W[s][r] = V_b,low^dagger (alpha_r 2^-k g * phi_r)
//   stage C  (tile, high bits)   grad_r += sum_s V_b,high^dagger W[s][r]
// Stage B holds all R atoms of a chunk on chip, so p, g and the adjoint are
// fused; stages A and C amortise the psi read and the gradient
// read-modify-write over the S settings of a batch.  All reductions are
// written to per-work-group slots and summed in a fixed order (deterministic).
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
// Low-stage LDS: per atom a real and an imaginary transpose plane of Upad
// entries; the |phi|^2 table [R][Upad] and the sensitivity row [Upad] live in
// the same space (they are never live together with a transpose); then one
// double per thread for the reductions.
size_t lo_lds_bytes(const Geometry& g) {
  const size_t U = (size_t)1 << g.n_lo;
  const size_t Upad = U + (U >> 5);
  const size_t nthr = (size_t)g.R << (g.n_lo - g.logv_lo);
  const size_t planes = ((2 * (size_t)g.R * Upad * g.elem) + 15) & ~(size_t)15;
  return planes + nthr * sizeof(double);
}

// Transpose the registers of a thread between two layouts through LDS; the
// real and imaginary parts use separate planes (padded indexing; both
// layouts are compile-time).
template <int LOGV, int LO_FROM, int LO_TO, typename T>
__device__ __forceinline__ void lds_transpose(T (&x)[1 << LOGV], T (&y)[1 << LOGV], T* re, T* im, int tau) {
  T* rw = re + pad_base<LOGV, LO_FROM>(tau);
  T* iw = im + pad_base<LOGV, LO_FROM>(tau);
#pragma unroll
  for (int i = 0; i < (1 << LOGV); ++i) {
    rw[pad_off<LO_FROM>(i)] = x[i];
    iw[pad_off<LO_FROM>(i)] = y[i];
  }
  __syncthreads();
  const T* rr = re + pad_base<LOGV, LO_TO>(tau);
  const T* ir = im + pad_base<LOGV, LO_TO>(tau);
#pragma unroll
  for (int i = 0; i < (1 << LOGV); ++i) {
    x[i] = rr[pad_off<LO_TO>(i)];
    y[i] = ir[pad_off<LO_TO>(i)];
  }
  __syncthreads();
}

// Forward chain: layout 0 (already loaded) .. last, transforming each layout's new bits.
template <int K, typename CH, int LOGV, typename T>
__device__ __forceinline__ void fwd_chain(T (&x)[1 << LOGV], T (&y)[1 << LOGV], T* re, T* im, int tau, uint64_t pc) {
  if constexpr (K < CH::count()) {
    if constexpr (K > 0) lds_transpose<LOGV, CH::lo(K - 1), CH::lo(K)>(x, y, re, im, tau);
    xform<LOGV, false>(x, y, layout_codes<LOGV>(pc, CH::lo(K), CH::lo(K), CH::top(K), 0, 0));
    fwd_chain<K + 1, CH, LOGV>(x, y, re, im, tau, pc);
  }
}

// Adjoint chain: from the last layout back to layout 0.
template <int K, typename CH, int LOGV, typename T>
__device__ __forceinline__ void adj_chain(T (&x)[1 << LOGV], T (&y)[1 << LOGV], T* re, T* im, int tau, uint64_t pc) {
  xform<LOGV, true>(x, y, layout_codes<LOGV>(pc, CH::lo(K), CH::lo(K), CH::top(K), 0, 0));
  if constexpr (K > 0) {
    lds_transpose<LOGV, CH::lo(K), CH::lo(K - 1)>(x, y, re, im, tau);
    adj_chain<K - 1, CH, LOGV>(x, y, re, im, tau, pc);
  }
}

template <typename T, int N_LO, bool ADJ>
__global__ __launch_bounds__(512) void k_stage_lo(const LoArgs a) {
  using C2 = cx<T>;
  constexpr int LOGV = N_LO < 5 ? N_LO : 5;
  constexpr int V = 1 << LOGV;
  constexpr int U = 1 << N_LO;
  constexpr int UPAD = U + (U >> 5);
  constexpr int LOG_TA = N_LO - LOGV;
  constexpr int TA = 1 << LOG_TA;
  using CH = Chain<N_LO, LOGV>;
  constexpr int NL = CH::count();
  constexpr int LO0 = CH::lo(0);
  constexpr uint32_t CB = sizeof(C2);
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  const int atom = tid >> LOG_TA;
  const int tau = tid & (TA - 1);
  const long long D = a.D;
  const int per_set = (1 << a.n_hi) / a.cpw;
  const int s = blockIdx.x / per_set;
  const int hg = blockIdx.x - s * per_set;
  const int b = a.b0 + s;
  const uint64_t pc = uniform_u64(a.pc[b]);
  const int kb = nonz_count(pc, a.n);
  const T s2 = (T)ldexp(1.0, -kb);
  const long long slot = (long long)b * per_set + hg;
  const double Bd = (double)a.B;

  // LDS: per atom a real and an imaginary plane of UPAD entries (transposes).  The
  // |phi|^2 table [R][UPAD] and the sensitivity row g [UPAD] alias the first R+1 rows
  // of the planes (2R rows in all); barriers separate their uses from the transposes.
  T* planes = reinterpret_cast<T*>(smem);
  T* re = planes + (size_t)atom * 2 * UPAD;
  T* im = re + UPAD;
  T* qb = planes;
  T* gb = planes + (size_t)a.R * UPAD;
  double* red = reinterpret_cast<double*>(smem + (((2 * (size_t)a.R * UPAD * sizeof(T)) + 15) & ~(size_t)15));

  const T al = (T)a.alpha[atom];
  const uint32_t vbytes = (uint32_t)(((long long)(a.R - 1) * D + U) * CB);
  const uint32_t vo0 = (uint32_t)(((long long)atom * D + lay_pos<LOGV>(tau, 0, LO0)) * CB);
  double loss_acc = 0.0, h_acc = 0.0;

  for (int cc = 0; cc < a.cpw; ++cc) {
    const int h = hg * a.cpw + cc;
    const C2* sbase = reinterpret_cast<const C2*>(a.src) + (long long)s * a.src_set_stride + ((long long)h << N_LO);
    const rsrc_t rs = make_rsrc(sbase, vbytes);
    T x[V], y[V];
#pragma unroll
    for (int i = 0; i < V; ++i) {
      C2 t;
      bload(t, rs, vo0, (uint32_t)(i << LO0) * CB);
      x[i] = t.x;
      y[i] = t.y;
    }
    fwd_chain<0, CH, LOGV>(x, y, re, im, tau, pc);
    // Final layout is lo = 0: alpha_r |phi_r|^2 into LDS, reduced over atoms per outcome.
    T* qrow = qb + (size_t)atom * UPAD + pad_base<LOGV, 0>(tau);
#pragma unroll
    for (int i = 0; i < V; ++i) qrow[pad_off<0>(i)] = al * (x[i] * x[i] + y[i] * y[i]);
    __syncthreads();
    for (int u = tid; u < U; u += nthr) {
      T p = 0;
      for (int r = 0; r < a.R; ++r) p += qb[(size_t)r * UPAD + pad32(u)];
      p *= s2;
      const long long gi = (long long)b * D + ((long long)h << N_LO) + u;
      if (a.probs) reinterpret_cast<T*>(a.probs)[gi] = p;
      T g = 0;
      if (a.grad_p) {
        g = reinterpret_cast<const T*>(a.grad_p)[gi];
      } else if (a.loss_kind == 0) {
        const double f = (double)a.freqs[gi];
        if (f > 0.0) {
          const double piv = (double)p / Bd + a.eps;
          loss_acc -= (f / Bd) * log(piv);
          g = (T)(-(f / Bd) / piv / Bd);
        }
      } else if (a.loss_kind == 1) {
        const double rr = ((double)p - (double)a.freqs[gi]) / Bd;
        loss_acc += 0.5 * rr * rr;
        g = (T)(rr / Bd);
      }
      if (a.gneg) reinterpret_cast<T*>(a.gneg)[gi] = -g;
      if (ADJ) gb[pad32(u)] = g * s2;
    }
    __syncthreads();
    if (ADJ) {
      T hl = 0;
#pragma unroll
      for (int i = 0; i < V; ++i) {
        const T gv = gb[pad_base<LOGV, 0>(tau) + pad_off<0>(i)];
        hl += gv * (x[i] * x[i] + y[i] * y[i]);
        const T sc = al * gv;
        x[i] *= sc;
        y[i] *= sc;
      }
      h_acc += (double)hl;
      __syncthreads();  // every thread has read g before the planes are reused
      adj_chain<NL - 1, CH, LOGV>(x, y, re, im, tau, pc);
      C2* dbase = reinterpret_cast<C2*>(a.dst) + (long long)s * a.R * D + ((long long)h << N_LO);
      const rsrc_t rd = make_rsrc(dbase, vbytes);
#pragma unroll
      for (int i = 0; i < V; ++i) bstore(C2{x[i], y[i]}, rd, vo0, (uint32_t)(i << LO0) * CB);
      __syncthreads();
    }
  }
  if (a.part == nullptr) return;
  if (ADJ) {
    red[tid] = h_acc;
    __syncthreads();
    for (int st = TA >> 1; st > 0; st >>= 1) {
      if (tau < st) red[tid] += red[tid + st];
      __syncthreads();
    }
    if (tau == 0) a.part[(long long)(1 + atom) * a.nslots + slot] = red[tid];
    __syncthreads();
  }
  if (a.grad_p == nullptr && a.loss_kind != 2) {
    red[tid] = loss_acc;
    __syncthreads();
    int np2 = 1;
    while (np2 < nthr) np2 <<= 1;
    for (int st = np2 >> 1; st > 0; st >>= 1) {
      if (tid < st && tid + st < nthr) red[tid] += red[tid + st];
      __syncthreads();
    }
    if (tid == 0) a.part[slot] = red[0];
  }
}

template <typename T, int N_LO>
static hipError_t launch_lo_n(const Geometry& g, const LoArgs& a, int S, bool adjoint, hipStream_t st) {
  constexpr int LOGV = N_LO < 5 ? N_LO : 5;
  const int nthr = g.R << (N_LO - LOGV);
  const size_t lds = lo_lds_bytes(g);
  const unsigned grid = (unsigned)(S * g.items_per_setting);
  if (adjoint) {
    hipFuncSetAttribute(reinterpret_cast<const void*>(&k_stage_lo<T, N_LO, true>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    k_stage_lo<T, N_LO, true><<<grid, nthr, lds, st>>>(a);
  } else {
    hipFuncSetAttribute(reinterpret_cast<const void*>(&k_stage_lo<T, N_LO, false>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    k_stage_lo<T, N_LO, false><<<grid, nthr, lds, st>>>(a);
  }
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_lo_v(const Geometry& g, const LoArgs& a, int S, bool adjoint, hipStream_t st) {
  switch (g.n_lo) {
    case 1: return launch_lo_n<T, 1>(g, a, S, adjoint, st);
    case 2: return launch_lo_n<T, 2>(g, a, S, adjoint, st);
    case 3: return launch_lo_n<T, 3>(g, a, S, adjoint, st);
    case 4: return launch_lo_n<T, 4>(g, a, S, adjoint, st);
    case 5: return launch_lo_n<T, 5>(g, a, S, adjoint, st);
    case 6: return launch_lo_n<T, 6>(g, a, S, adjoint, st);
    case 7: return launch_lo_n<T, 7>(g, a, S, adjoint, st);
    case 8: return launch_lo_n<T, 8>(g, a, S, adjoint, st);
    case 9: return launch_lo_n<T, 9>(g, a, S, adjoint, st);
    case 10: return launch_lo_n<T, 10>(g, a, S, adjoint, st);
    case 11: return launch_lo_n<T, 11>(g, a, S, adjoint, st);
    case 12: return launch_lo_n<T, 12>(g, a, S, adjoint, st);
    case 13: return launch_lo_n<T, 13>(g, a, S, adjoint, st);
    case 14: return launch_lo_n<T, 14>(g, a, S, adjoint, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_stage_lo(const Geometry& g, const LoArgs& a, int S, bool adjoint, hipStream_t st) {
  return g.elem == 4 ? launch_lo_v<float>(g, a, S, adjoint, st) : launch_lo_v<double>(g, a, S, adjoint, st);
}

// ------------------------------------------------------------------ stages A and C
size_t hi_lds_bytes(const Geometry& g) {
  const size_t N = (size_t)1 << g.t;
  return (N + (N >> 5)) * 2 * (size_t)g.elem;
}

// Offset (elements from the tile origin) of tile position lam: tile bits below c
// are columns (index bits 0..c-1), the rest are rows (index bits n_lo..).
__device__ __forceinline__ uint32_t tile_off(uint32_t lam, int c, int n_lo) {
  return ((lam >> c) << n_lo) | (lam & ((1u << c) - 1u));
}

// Mask of the register bits of layout `lo` that are tile rows (qubits of the
// high pass) and are transformed in this layout: bits [max(lo, c), top).
constexpr uint32_t rows_mask(int lo, int c, int top) {
  uint32_t m = 0;
  for (int k = 0; k < 5; ++k)
    if (lo + k >= c && lo + k < top) m |= 1u << k;
  return m;
}

template <int TB, int N_HI, bool ADJ>
__global__ __launch_bounds__(512) void k_stage_hi(const HiArgs a) {
  using T = float;
  using C2 = float2;
  constexpr int LOGV = 5;
  constexpr int V = 1 << LOGV;
  constexpr int C = TB - N_HI;           // column bits of the tile
  constexpr int LO0 = TB - LOGV;
  constexpr bool TWO = C < LO0;          // rows reach below the first layout
  constexpr int LO1 = TB - 2 * LOGV > 0 ? TB - 2 * LOGV : 0;
  constexpr int LOF = TWO ? LO1 : LO0;
  constexpr uint32_t M0 = rows_mask(LO0, C, TB);
  constexpr uint32_t M1 = rows_mask(LO1, C, LO0);
  constexpr int NPAD = (1 << TB) + (1 << (TB - 5));
  constexpr uint32_t CB = sizeof(C2);
  static_assert(!TWO || TB - 2 * LOGV >= 0 || C >= 0, "tile layouts");
  extern __shared__ __align__(16) unsigned char smem[];
  T* re = reinterpret_cast<T*>(smem);
  T* im = re + NPAD;
  const int tid = threadIdx.x;
  const int n_lo = a.n_lo;
  const int ncb = 1 << (n_lo - C);
  const int r = blockIdx.x / ncb;
  const int cb = blockIdx.x - r * ncb;
  const long long D = a.D;
  const long long origin = (long long)r * D + ((long long)cb << C);
  const uint32_t vbytes = (uint32_t)((D - ((long long)cb << C)) * CB);
  const uint32_t vo0 = tile_off(lay_pos<LOGV>(tid, 0, LO0), C, n_lo) * CB;
  const uint32_t vof = tile_off(lay_pos<LOGV>(tid, 0, LOF), C, n_lo) * CB;

  if (!ADJ) {
    const rsrc_t rs = make_rsrc(reinterpret_cast<const C2*>(a.src) + origin, vbytes);
    T kx[V], ky[V];
#pragma unroll
    for (int i = 0; i < V; ++i) {
      C2 t;
      bload(t, rs, vo0, tile_off((uint32_t)i << LO0, C, n_lo) * CB);
      kx[i] = t.x;
      ky[i] = t.y;
    }
    for (int s = 0; s < a.S; ++s) {
      const uint64_t pc = uniform_u64(a.pc[a.b0 + s]);
      T x[V], y[V];
#pragma unroll
      for (int i = 0; i < V; ++i) {
        x[i] = kx[i];
        y[i] = ky[i];
      }
      xform_uniform<LOGV, false, M0>(x, y, layout_codes<LOGV>(pc, LO0, LO0, TB, C, n_lo));
      if constexpr (TWO) {
        lds_transpose<LOGV, LO0, LO1>(x, y, re, im, tid);
        xform_uniform<LOGV, false, M1>(x, y, layout_codes<LOGV>(pc, LO1, LO1, LO0, C, n_lo));
      }
      const rsrc_t rx = make_rsrc(reinterpret_cast<C2*>(a.dst) + (long long)s * a.R * D + origin, vbytes);
#pragma unroll
      for (int i = 0; i < V; ++i) bstore(C2{x[i], y[i]}, rx, vof, tile_off((uint32_t)i << LOF, C, n_lo) * CB);
    }
  } else {
    T ax[V], ay[V];
#pragma unroll
    for (int i = 0; i < V; ++i) ax[i] = ay[i] = T(0);
    for (int s = 0; s < a.S; ++s) {
      const uint64_t pc = uniform_u64(a.pc[a.b0 + s]);
      const rsrc_t rw = make_rsrc(reinterpret_cast<const C2*>(a.src) + (long long)s * a.R * D + origin, vbytes);
      T x[V], y[V];
#pragma unroll
      for (int i = 0; i < V; ++i) {
        C2 t;
        bload(t, rw, vo0, tile_off((uint32_t)i << LO0, C, n_lo) * CB);
        x[i] = t.x;
        y[i] = t.y;
      }
      xform_uniform<LOGV, true, M0>(x, y, layout_codes<LOGV>(pc, LO0, LO0, TB, C, n_lo));
      if constexpr (TWO) {
        lds_transpose<LOGV, LO0, LO1>(x, y, re, im, tid);
        xform_uniform<LOGV, true, M1>(x, y, layout_codes<LOGV>(pc, LO1, LO1, LO0, C, n_lo));
      }
#pragma unroll
      for (int i = 0; i < V; ++i) {
        ax[i] += x[i];
        ay[i] += y[i];
      }
    }
    const rsrc_t rg = make_rsrc(reinterpret_cast<C2*>(a.dst) + origin, vbytes);
#pragma unroll
    for (int i = 0; i < V; ++i) {
      const uint32_t so = tile_off((uint32_t)i << LOF, C, n_lo) * CB;
      if (!a.first) {
        C2 t;
        bload(t, rg, vof, so);
        ax[i] += t.x;
        ay[i] += t.y;
      }
      bstore(C2{ax[i], ay[i]}, rg, vof, so);
    }
  }
}

template <int TB, int N_HI>
static hipError_t launch_hi_n(const Geometry& g, const HiArgs& a, bool adjoint, hipStream_t st) {
  const int nthr = 1 << (TB - 5);
  const size_t lds = hi_lds_bytes(g);
  const unsigned grid = (unsigned)(g.R << (g.n_lo - g.c));
  if (adjoint) {
    hipFuncSetAttribute(reinterpret_cast<const void*>(&k_stage_hi<TB, N_HI, true>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    k_stage_hi<TB, N_HI, true><<<grid, nthr, lds, st>>>(a);
  } else {
    hipFuncSetAttribute(reinterpret_cast<const void*>(&k_stage_hi<TB, N_HI, false>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    k_stage_hi<TB, N_HI, false><<<grid, nthr, lds, st>>>(a);
  }
  return hipGetLastError();
}

// Supported (tile bits, high bits) pairs of the FP32 path: n in 11..20 with the
// low-stage sizes chosen by the host (n_lo >= 10).
hipError_t launch_stage_hi(const Geometry& g, const HiArgs& a, bool adjoint, hipStream_t st) {
  if (g.elem != 4) return hipErrorInvalidValue;
#define QST_HI(TBv, NHv) \
  if (g.t == TBv && g.n_hi == NHv) return launch_hi_n<TBv, NHv>(g, a, adjoint, st);
  QST_HI(14, 1) QST_HI(14, 2) QST_HI(14, 3) QST_HI(14, 4) QST_HI(14, 5)
  QST_HI(14, 6) QST_HI(14, 7) QST_HI(14, 8) QST_HI(14, 9) QST_HI(14, 10)
  QST_HI(13, 1) QST_HI(13, 2) QST_HI(13, 3) QST_HI(12, 1) QST_HI(12, 2) QST_HI(11, 1)
#undef QST_HI
  return hipErrorInvalidValue;
}


// ------------------------------------------------------------------ sum over settings (no high bits)
template <typename T>
__global__ void k_sum_settings(const cx<T>* __restrict__ W, int S, long long RD, cx<T>* __restrict__ grad, int first) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < RD; e += (long long)gridDim.x * blockDim.x) {
    cx<T> acc{0, 0};
    for (int s = 0; s < S; ++s) {
      const cx<T> w = W[(long long)s * RD + e];
      acc.x += w.x;
      acc.y += w.y;
    }
    if (first) {
      grad[e] = acc;
    } else {
      cx<T> x = grad[e];
      grad[e] = cx<T>{x.x + acc.x, x.y + acc.y};
    }
  }
}

hipError_t launch_sum_settings(const Geometry& g, const void* W, int S, void* grad, int first, hipStream_t st) {
  const long long RD = (long long)g.R * g.D;
  const int bs = 256;
  long long nb = (RD + bs - 1) / bs;
  if (nb > 8192) nb = 8192;
  if (g.elem == 4)
    k_sum_settings<float><<<(unsigned)nb, bs, 0, st>>>(reinterpret_cast<const float2*>(W), S, RD,
                                                        reinterpret_cast<float2*>(grad), first);
  else
    k_sum_settings<double><<<(unsigned)nb, bs, 0, st>>>(reinterpret_cast<const double2*>(W), S, RD,
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
    if (a.probs) reinterpret_cast<float*>(a.probs)[gi] = p;
    if (a.grad_p) {
      g = reinterpret_cast<const float*>(a.grad_p)[gi];
    } else if (a.loss_kind == 0) {
      const double f = (double)a.freqs[gi];
      if (f > 0.0) {
        const double piv = (double)p / Bd + a.eps;
        loss = -(f / Bd) * log(piv);
        g = (float)(-(f / Bd) / piv / Bd);
      }
    } else if (a.loss_kind == 1) {
      const double rr = ((double)p - (double)a.freqs[gi]) / Bd;
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

}  // namespace qst
