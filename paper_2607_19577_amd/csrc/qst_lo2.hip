// Two-sweep low stage: the low pass of the staged path for chunks whose atoms do not fit one
// work-group together (R 2^n_lo > 2^14).  A work-group holds one atom's part of a chunk
// (2^n_lo amplitudes of one setting) at a time and loops over the atoms twice:
//
//   sweep 1: phi_r = (low-bit rotation) X_r for r = 0..R-1, acc += alpha_r |phi_r|^2 in
//            registers (every atom's last layout puts the same outcomes in the same thread);
//            then p = 2^-k acc (+ base), the loss terms (eq. qst-loss) and g = dL/dp
//            (eq. likelihood-ratio-vector), kept in registers as G = 2^-k g;
//   sweep 2: phi_r again, the weight-gradient term sum G |phi_r|^2 (eq. weight-gradient),
//            alpha_r G phi_r through the adjoint low-bit rotation into W
//            (eq. atom-wirtinger-gradient; the high bits follow in the adjoint tile stage).
//
// X is read twice and W written once (24 B per (setting, atom) amplitude) where a three-pass
// schedule would move 48 (the middle pass reads and writes X and W once more); the price is
// a third rotation of the low bits.  With n_lo = n - 10 every state up to n = 24 keeps two
// tile passes.  Pauli settings and dense data, FP32 arithmetic, X and W in FP32 or BF16;
// n_lo = 10..14.
#include "qst_stages.hpp"

namespace qst {

namespace {

// One atom's 2^NB amplitudes per work-group: 32 per thread (16 at NB = 10, so that a
// work-group is at least one wavefront).
constexpr int lo2_logv(int nb) { return nb <= 10 ? 4 : 5; }
template <int NB>
constexpr int lo2_threads() {
  return 1 << (NB - lo2_logv(NB));
}

}  // namespace

template <int NB, bool ADJ, bool H16>
__global__ __launch_bounds__(lo2_threads<NB>()) void k_stage_lo2(const LoArgs a) {
  constexpr int LOGV = lo2_logv(NB);
  constexpr int V = 1 << LOGV;
  constexpr int LOG_TA = NB - LOGV;
  constexpr int NT = 1 << LOG_TA;
  constexpr int NW = NT >= 64 ? NT / 64 : 1;  // wavefronts per work-group
  constexpr int U = 1 << NB;
  constexpr int UPAD = U + (U >> 5);
  constexpr bool WL = LOG_TA <= 6;
  using CH = Chain<NB, LOGV>;
  constexpr int NL = CH::count();
  constexpr int LO0 = CH::lo(0);
  constexpr uint32_t CBH = H16 ? 4u : 8u;  // bytes per complex of X and W
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  float* re = reinterpret_cast<float*>(smem);
  float* im = WL ? re : re + UPAD;
  // per-wavefront weight-gradient sums [NW][R], then one double per thread for the loss
  double* hw = reinterpret_cast<double*>(smem + ((((size_t)(WL ? 1 : 2) * UPAD * 4) + 15) & ~(size_t)15));
  double* red = hw + (size_t)NW * a.R;
  const uint32_t pos0 = (uint32_t)lay_pos<LOGV>(tid, 0, LO0);
  auto off0 = [](int i) { return (uint32_t)(i << LO0); };
  const long long D = a.D;
  const float inv_b = (float)(1.0 / (double)a.B);
  const float eps_f = (float)a.eps;
  const float* gp = reinterpret_cast<const float*>(a.grad_p);
  const float* pbp = reinterpret_cast<const float*>(a.pbase);

  for (int r = tid; r < NW * a.R; r += NT) hw[r] = 0.0;
  __syncthreads();
  double loss_acc = 0.0;

  for (int c = blockIdx.x; c < a.nchunks; c += gridDim.x) {
#pragma clang fp contract(off)
    const int s = c >> a.n_hi;
    const int h = c & ((1 << a.n_hi) - 1);
    const int b = a.b0 + s;
    const uint64_t pc = load_code(a.pc, b);
    const float s2 = (float)ldexp(1.0, -nonz_count(pc, a.n));
    // Atom r's part of the chunk: element l at (h << xb) + xpos(l) of the atom's vector in X,
    // index bits [xb, NB) of l stored above the high bits (xb = NB: plain order); likewise W.
    const int xb = NB - a.x_up, wb = NB - a.w_up;
    auto xpos = [&](uint32_t l) { return ((l >> xb) << (a.n_hi + xb)) | (l & ((1u << xb) - 1u)); };
    auto wpos = [&](uint32_t l) { return ((l >> wb) << (a.n_hi + wb)) | (l & ((1u << wb) - 1u)); };
    const long long cbase = (long long)s * a.src_set_stride + ((long long)h << xb);
    const uint32_t xext = (uint32_t)((D - ((long long)h << xb)) * CBH);
    auto load = [&](int r, float (&x)[V], float (&y)[V]) __attribute__((always_inline)) {
      const rsrc_t rs = make_rsrc(reinterpret_cast<const unsigned char*>(a.src) + (cbase + (long long)r * D) * CBH, xext);
#pragma unroll
      for (int i = 0; i < V; ++i) ld_cs<H16>(x[i], y[i], rs, xpos(pos0) * CBH, xpos(off0(i)) * CBH);
    };
    float acc[V];
#pragma unroll
    for (int i = 0; i < V; ++i) acc[i] = 0.0f;
    for (int r = 0; r < a.R; ++r) {
      float x[V], y[V];
      load(r, x, y);
      fwd_chain<0, CH, WL, false, LOGV>(x, y, re, im, tid, pc, nullptr);
      const float al = (float)a.alpha[r];
#pragma unroll
      for (int i = 0; i < V; ++i) acc[i] = fma(al, fma(x[i], x[i], y[i] * y[i]), acc[i]);
    }
    // This thread's outcomes (last layout lo = 0): u = (tid << LOGV) + i of the chunk.
    const long long row = (long long)b * D + ((long long)h << NB) + ((long long)tid << LOGV);
    float G[V];
#pragma unroll
    for (int i = 0; i < V; ++i) {
      float p = acc[i] * s2;
      if (pbp) p += pbp[row + i];
      if (a.probs) reinterpret_cast<float*>(a.probs)[row + i] = p;
      float g = 0.0f;
      if (gp) {
        g = gp[row + i];
      } else if (a.loss_kind == 0) {
        const float d = a.freqs[row + i];
        if (d > 0.0f) {
          // each term in FP32 (hardware log2 and reciprocal), summed in FP64
          const float fb = d * inv_b;
          const float piv = fmaf(p, inv_b, eps_f);
          loss_acc -= (double)(fb * (__builtin_amdgcn_logf(piv) * 0.693147180559945309f));
          g = -(fb * inv_b) * __builtin_amdgcn_rcpf(piv);
        }
      } else if (a.loss_kind == 1) {
        const float rr = (p - a.freqs[row + i]) * inv_b;
        loss_acc += (double)(0.5f * rr * rr);
        g = rr * inv_b;
      }
      if (a.gneg) reinterpret_cast<float*>(a.gneg)[row + i] = -g;
      G[i] = g * s2;
    }
    if constexpr (ADJ) {
      const long long wbase = (long long)s * a.R * D + ((long long)h << wb);
      const uint32_t wext = (uint32_t)((D - ((long long)h << wb)) * CBH);
      // atoms in reverse order: the last ones read by sweep 1 may still be in L2 (n=22, R=16:
      // 162.1 against 165.8 ms per step in this stage)
      for (int r = a.R - 1; r >= 0; --r) {
        float x[V], y[V];
        load(r, x, y);
        fwd_chain<0, CH, WL, false, LOGV, false>(x, y, re, im, tid, pc, nullptr);
        const float al = (float)a.alpha[r];
        float hl = 0.0f;
#pragma unroll
        for (int i = 0; i < V; ++i) {
          hl = fma(G[i], fma(x[i], x[i], y[i] * y[i]), hl);
          const float sc = al * G[i];
          x[i] *= sc;
          y[i] *= sc;
        }
        // weight-gradient term of atom r: a fixed-order tree over the wavefront's lanes, then
        // one slot per wavefront (no two wavefronts write the same slot)
        double hd = (double)hl;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) hd += __shfl_xor(hd, o);
        if (lane == 0) hw[wave * a.R + r] += hd;
        adj_chain<NL - 1, CH, WL, false, LOGV>(x, y, re, im, tid, pc, nullptr);
        const rsrc_t rw = make_rsrc(reinterpret_cast<unsigned char*>(a.dst) + (wbase + (long long)r * D) * CBH, wext);
#pragma unroll
        for (int i = 0; i < V; ++i) st_cs<H16>(x[i], y[i], rw, wpos(pos0) * CBH, wpos(off0(i)) * CBH);
      }
    }
  }
  // Partials of this work-group: loss in row 0, h_r in rows 1..R (zero if it had no chunk).
  if (a.part == nullptr) return;
  const long long slot = a.slot_base + blockIdx.x;
  red[tid] = loss_acc;
  __syncthreads();
  for (int st = NT >> 1; st > 0; st >>= 1) {
    if (tid < st) red[tid] += red[tid + st];
    __syncthreads();
  }
  if (tid == 0) a.part[slot] = red[0];
  if (ADJ) {
    for (int r = tid; r < a.R; r += NT) {
      double v = 0.0;
      for (int w = 0; w < NW; ++w) v += hw[w * a.R + r];
      a.part[(long long)(1 + r) * a.nslots + slot] = v;
    }
  }
}

size_t lo2_lds_bytes(const Geometry& g) {
  const size_t U = (size_t)1 << g.n_lo;
  const size_t UPAD = U + (U >> 5);
  const int logv = lo2_logv(g.n_lo);
  const size_t nt = (size_t)1 << (g.n_lo - logv);
  const size_t nw = nt >= 64 ? nt / 64 : 1;
  const bool wl = g.n_lo - logv <= 6;
  return ((((wl ? 1 : 2) * UPAD * 4) + 15) & ~(size_t)15) + nw * (size_t)g.R * 8 + nt * 8;
}

namespace {

template <int NB, bool ADJ, bool H16>
hipError_t launch_lo2_n(const Geometry& g, const LoArgs& a, hipStream_t st) {
  const size_t lds = lo2_lds_bytes(g);
  const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_stage_lo2<NB, ADJ, H16>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  k_stage_lo2<NB, ADJ, H16><<<g.grid_lo, lo2_threads<NB>(), lds, st>>>(a);
  return hipGetLastError();
}

template <int NB, bool H16>
int occupancy_lo2_n(const Geometry& g) {
  const size_t lds = lo2_lds_bytes(g);
  const void* f = reinterpret_cast<const void*>(&k_stage_lo2<NB, true, H16>);
  if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) return 1;
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_stage_lo2<NB, true, H16>, lo2_threads<NB>(), lds) !=
      hipSuccess)
    return 1;
  return blocks > 0 ? blocks : 1;
}

}  // namespace

hipError_t launch_stage_lo2(const Geometry& g, const LoArgs& a, bool adjoint, hipStream_t st) {
  if (g.elem != 4 || g.gen || a.fidx != nullptr || a.R < 1 || a.nchunks < 0 || g.grid_lo < 1)
    return hipErrorInvalidValue;
#define QST_LO2(NBv)                                                                              \
  if (g.n_lo == NBv) {                                                                            \
    if (g.h16) return adjoint ? launch_lo2_n<NBv, true, true>(g, a, st) : launch_lo2_n<NBv, false, true>(g, a, st); \
    return adjoint ? launch_lo2_n<NBv, true, false>(g, a, st) : launch_lo2_n<NBv, false, false>(g, a, st);         \
  }
  QST_LO2(10) QST_LO2(11) QST_LO2(12) QST_LO2(13) QST_LO2(14)
#undef QST_LO2
  return hipErrorInvalidValue;
}

int lo2_occupancy(const Geometry& g) {
  switch (g.n_lo) {
    case 10: return g.h16 ? occupancy_lo2_n<10, true>(g) : occupancy_lo2_n<10, false>(g);
    case 11: return g.h16 ? occupancy_lo2_n<11, true>(g) : occupancy_lo2_n<11, false>(g);
    case 12: return g.h16 ? occupancy_lo2_n<12, true>(g) : occupancy_lo2_n<12, false>(g);
    case 13: return g.h16 ? occupancy_lo2_n<13, true>(g) : occupancy_lo2_n<13, false>(g);
    case 14: return g.h16 ? occupancy_lo2_n<14, true>(g) : occupancy_lo2_n<14, false>(g);
    default: return 1;
  }
}

}  // namespace qst
