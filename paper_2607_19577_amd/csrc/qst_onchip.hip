// On-chip path for states of 2^11 .. 2^14 amplitudes (FP32, Pauli settings, dense data).
//
// The vector of one (setting, atom) pair -- at most 2^14 complex values, 128 KiB --
// fits one work-group's registers, so its whole basis rotation V_b psi_r (all n
// qubits) runs on chip.  When all R atoms of a setting do not fit at once
// (R 2^n > 2^14), the staged path round-trips the intermediates X and W through HBM
// once per setting and atom; here they are recomputed instead:
//
//   pass F  (item = instance, group of settings; one setting per vector):
//           for r = 0..R-1: phi = V_b psi_r, acc += alpha_r |phi|^2   (the atom sum in
//           registers: every atom's final layout puts the same outcomes in the same
//           thread); p = 2^-k acc (+ base); loss terms (eq. qst-loss) and the
//           sensitivity g = dL/dp (eq. likelihood-ratio-vector); writes 2^-k g to G.
//   pass A  (item = instance, tile of atoms, slice of settings; one atom per vector):
//           psi_r is kept in registers; per setting phi = V_b psi_r again, the
//           weight-gradient partial sum 2^-k g |phi|^2 (eq. weight-gradient), then
//           alpha_r 2^-k g * phi through the adjoint rotation V_b^dagger, summed over
//           the slice in registers (eq. atom-wirtinger-gradient).  One partial gradient
//           per slice goes to HBM; k_oc_sum adds the slices in a fixed order.
//
// HBM traffic per call: the frequencies (read), G (written once, read by the atom
// tiles of a slice, mostly from L2), the slice partials and the atoms -- about
// 4 + 4 + 4 B per outcome and setting plus 16 B per partial amplitude, instead of the
// staged path's 32 B per (setting, atom) amplitude.  The price is a third rotation per
// (setting, atom): the path is bound by vector arithmetic and LDS transposes.
//
// Every wavefront holds part of exactly one vector (2^(n-5) >= 64 threads per vector),
// so setting-dependent branches (Z bits) stay uniform per wavefront.
#include "qst_stages.hpp"

namespace qst {

namespace {

// Threads per work-group with 2^LOGV values per thread: one vector of 2^(NB-LOGV) threads, or
// 256 threads holding several vectors.
template <int NB, int LOGV>
constexpr int oc_threads() {
  return (1 << (NB - LOGV)) > 256 ? (1 << (NB - LOGV)) : 256;
}

// Instance of item `i` of a launch over instances [k0, k1) (first item of instance k at
// first(k)): linear search, uniform.
template <typename F>
__device__ __forceinline__ int oc_find(int k0, int k1, int i, F first) {
  int k = k0;
  while (k + 1 < k1 && i >= first(k + 1)) ++k;
  return k;
}

__device__ __forceinline__ float4 ld_f4(const float* p) { return *reinterpret_cast<const float4*>(p); }

}  // namespace

// ------------------------------------------------------------------ pass F
template <int NB, int LOGV>
__global__ __launch_bounds__((oc_threads<NB, LOGV>())) void k_oc_fwd(const OcInst* __restrict__ tab, int k0, int k1,
                                                                int total) {
  constexpr int V = 1 << LOGV;
  constexpr int LOG_TA = NB - LOGV;
  constexpr int TA = 1 << LOG_TA;
  constexpr int NT = oc_threads<NB, LOGV>();
  constexpr int VPW = NT / TA;
  constexpr int U = 1 << NB;
  constexpr int UPAD = U + (U >> 5);
  constexpr bool WL = LOG_TA <= 6;
  using CH = Chain<NB, LOGV>;
  constexpr int LO0 = CH::lo(0);
  static_assert(TA >= 64, "one vector per wavefront at least");
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;
  const int vec = tid >> LOG_TA;
  const int tau = tid & (TA - 1);
  float* re = reinterpret_cast<float*>(smem) + (size_t)vec * (WL ? 1 : 2) * UPAD;
  float* im = WL ? re : re + UPAD;
  double* red = reinterpret_cast<double*>(smem + (((size_t)VPW * (WL ? 1 : 2) * UPAD * 4 + 15) & ~(size_t)15));
  const uint32_t pos0 = (uint32_t)lay_pos<LOGV>(tau, 0, LO0);
  const uint32_t vo0 = pos0 * 8u;
  auto off0 = [](int i) { return (uint32_t)(i << LO0); };

  for (int item = blockIdx.x; item < total; item += gridDim.x) {
#pragma clang fp contract(off)
    const int k = oc_find(k0, k1, item, [&](int kk) { return tab[kk].itemF0; });
    const OcInst& a = tab[k];
    const int j = item - a.itemF0;
    const int s_beg = j * a.sF;
    const int s_end = min(a.B, s_beg + a.sF);
    const int R = a.R;
    const long long D = 1ll << NB;
    const float inv_b = (float)(1.0 / (double)a.B);
    const float eps_f = (float)a.eps;
    const rsrc_t rs = make_rsrc(a.atoms, (uint32_t)((long long)R * D * 8));
    double loss_acc = 0.0;
    for (int sb = s_beg; sb < s_end; sb += VPW) {
      const int s = sb + vec;
      const bool valid = s < s_end;
      const int b = valid ? s : s_beg;  // a spare vector repeats a setting and writes nothing
      const uint64_t pc = load_code(a.pc, b);
      const uint32_t ym = ymask_of(pc, NB);
      const float s2 = (float)ldexp(1.0, -nonz_count(pc, NB));
      float acc[V];
#pragma unroll
      for (int i = 0; i < V; ++i) acc[i] = 0.0f;
      // One atom at a time (no prefetch: the registers go to occupancy, and the other
      // wavefronts of the compute unit cover the load latency).
      for (int r = 0; r < R; ++r) {
        float x[V], y[V];
        const uint32_t base = (uint32_t)((long long)r * D * 8);
#pragma unroll
        for (int i = 0; i < V; ++i) bload2(x[i], y[i], rs, vo0 + base, off0(i) * 8u);
        const float al = (float)a.alpha[r];
        apply_phase<false, LOGV>(x, y, pos0, ym, off0);
        fwd_chain<0, CH, WL, false, LOGV>(x, y, re, im, tau, pc, nullptr);
#pragma unroll
        for (int i = 0; i < V; ++i) acc[i] = fma(al, fma(x[i], x[i], y[i] * y[i]), acc[i]);
      }
      // The atom sum goes through this vector's LDS plane so that consecutive lanes take
      // consecutive outcomes u = tau + e 2^(n-LOGV): the data row and the outputs are then read
      // and written in whole lines.  (The last rotation's transposes are done with the plane.)
      {
        float* prow = re + pad_base<LOGV, 0>(tau);
#pragma unroll
        for (int i = 0; i < V; ++i) prow[pad_off<0>(i)] = acc[i];
      }
      if constexpr (WL)
        wave_sync();
      else
        __syncthreads();
      const long long row = (long long)b * D;
      const bool gen = a.grad_p != nullptr;
      const bool data = a.freqs != nullptr && !gen;
#pragma unroll
      for (int e0 = 0; e0 < V; e0 += 8) {
        float d[8], pb[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const long long u = tau + (long long)(e0 + e) * TA;
          d[e] = data ? a.freqs[row + u] : 0.0f;
          pb[e] = a.pbase != nullptr ? a.pbase[row + u] : 0.0f;
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int u = tau + (e0 + e) * TA;
          float pv = re[pad32(u)] * s2;
          if (a.pbase != nullptr) pv += pb[e];
          float g = 0.0f;
          if (a.loss_kind == 0) {
            if (d[e] > 0.0f) {
              // each term in FP32 (hardware log2 and reciprocal), summed in FP64
              const float fb = d[e] * inv_b;
              const float piv = fmaf(pv, inv_b, eps_f);
              if (valid) loss_acc -= (double)(fb * (__builtin_amdgcn_logf(piv) * 0.693147180559945309f));
              g = -(fb * inv_b) * __builtin_amdgcn_rcpf(piv);
            }
          } else if (a.loss_kind == 1) {
            const float rr = (pv - d[e]) * inv_b;
            if (valid) loss_acc += (double)(0.5f * rr * rr);
            g = rr * inv_b;
          }
          if (valid) {
            if (a.probs != nullptr) a.probs[row + u] = pv;
            if (a.G != nullptr) a.G[row + u] = g * s2;
            if (a.gneg != nullptr) a.gneg[row + u] = -g;
          }
        }
      }
      if constexpr (WL)
        wave_sync();  // the plane's reads precede the next rotation's writes
      else
        __syncthreads();
    }
    // Loss partial of this item to slot j; weight-gradient rows of the slots pass A does not
    // write (j >= nA) are zeroed here, so every slot is defined.
    if (a.part != nullptr) {
      red[tid] = loss_acc;
      __syncthreads();
      for (int st = NT >> 1; st > 0; st >>= 1) {
        if (tid < st) red[tid] += red[tid + st];
        __syncthreads();
      }
      if (tid == 0) a.part[j] = red[0];
      if (j >= a.nA)
        for (int r = tid; r < R; r += NT) a.part[(long long)(1 + r) * a.nslots + j] = 0.0;
      __syncthreads();
    }
  }
}

// ------------------------------------------------------------------ pass A
template <int NB, int LOGV>
__global__ __launch_bounds__((oc_threads<NB, LOGV>()), (LOGV == 5 ? 2 : 4)) void k_oc_adj(
    const OcInst* __restrict__ tab, int k0, int k1, int total) {
  constexpr int V = 1 << LOGV;
  constexpr int LOG_TA = NB - LOGV;
  constexpr int TA = 1 << LOG_TA;
  constexpr int NT = oc_threads<NB, LOGV>();
  constexpr int VPW = NT / TA;
  constexpr int U = 1 << NB;
  constexpr int UPAD = U + (U >> 5);
  constexpr bool WL = LOG_TA <= 6;
  using CH = Chain<NB, LOGV>;
  constexpr int NL = CH::count();
  constexpr int LO0 = CH::lo(0);
  static_assert(TA >= 64, "one vector per wavefront at least");
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;
  const int vec = tid >> LOG_TA;
  const int tau = tid & (TA - 1);
  float* re = reinterpret_cast<float*>(smem) + (size_t)vec * (WL ? 1 : 2) * UPAD;
  float* im = WL ? re : re + UPAD;
  double* red = reinterpret_cast<double*>(smem + (((size_t)VPW * (WL ? 1 : 2) * UPAD * 4 + 15) & ~(size_t)15));
  const uint32_t pos0 = (uint32_t)lay_pos<LOGV>(tau, 0, LO0);
  const uint32_t vo0 = pos0 * 8u;
  auto off0 = [](int i) { return (uint32_t)(i << LO0); };

  for (int item = blockIdx.x; item < total; item += gridDim.x) {
#pragma clang fp contract(off)
    const int k = oc_find(k0, k1, item, [&](int kk) { return tab[kk].itemA0; });
    const OcInst& a = tab[k];
    const int j = item - a.itemA0;
    // Items map to (slice, atom tile) so that the tiles of one slice share j mod 8: work-groups
    // are dispatched to the eight XCDs in turn, so those tiles run on one XCD, close in time, and
    // the slice's rows of 2^-k dL/dp come from that XCD's L2 after the first tile's read.
    int slice, tile;
    {
      const int full = (a.nA / 8) * 8;  // slices in whole groups of eight
      if (j < full * a.ntile) {
        const int grp = j / (8 * a.ntile), rem = j - grp * 8 * a.ntile;
        slice = grp * 8 + (rem & 7);
        tile = rem >> 3;
      } else {
        const int jj = j - full * a.ntile;
        slice = full + jj / a.ntile;
        tile = jj - (slice - full) * a.ntile;
      }
    }
    const int R = a.R;
    const int r = tile * VPW + vec;
    const bool active = r < R;
    const long long D = 1ll << NB;
    const int s_beg = slice * a.sA;
    const int s_end = min(a.B, s_beg + a.sA);
    // psi_r is read again for every setting (from L2: the atoms of an instance are small);
    // atoms beyond the rank read zeros through the buffer bound.
    const rsrc_t rs = make_rsrc(a.atoms, (uint32_t)((long long)R * D * 8));
    const uint32_t abase = (uint32_t)((long long)(active ? r : R) * D * 8);
    const float al = active ? (float)a.alpha[r] : 0.0f;
    float ax[V], ay[V];
#pragma unroll
    for (int i = 0; i < V; ++i) ax[i] = ay[i] = 0.0f;
    double h_acc = 0.0;
    const bool gen = a.grad_p != nullptr;
    const float* gsrc = gen ? a.grad_p : a.G;
    for (int b = s_beg; b < s_end; ++b) {
      const uint64_t pc = load_code(a.pc, b);
      const uint32_t ym = ymask_of(pc, NB);
      const float s2 = (float)ldexp(1.0, -nonz_count(pc, NB));
      float x[V], y[V];
#pragma unroll
      for (int i = 0; i < V; ++i) bload2(x[i], y[i], rs, vo0 + abase, off0(i) * 8u);
      apply_phase<false, LOGV>(x, y, pos0, ym, off0);
      fwd_chain<0, CH, WL, false, LOGV, false>(x, y, re, im, tau, pc, nullptr);
      // this thread's outcomes (final layout lo = 0)
      const long long row = (long long)b * D + ((long long)tau << LOGV);
      float g[V];
#pragma unroll
      for (int q = 0; q < V / 4; ++q) {
        const float4 v = ld_f4(gsrc + row + 4 * q);
        g[4 * q] = v.x, g[4 * q + 1] = v.y, g[4 * q + 2] = v.z, g[4 * q + 3] = v.w;
      }
      float hl = 0.0f;
#pragma unroll
      for (int i = 0; i < V; ++i) {
        const float gv = gen ? g[i] * s2 : g[i];
        hl = fma(gv, fma(x[i], x[i], y[i] * y[i]), hl);
        const float sc = al * gv;
        x[i] *= sc;
        y[i] *= sc;
      }
      h_acc += (double)hl;
      // (the adjoint chain starts with the forward chain's last transpose reversed, which
      // touches only positions of this wavefront; its work-group transposes end with a
      // barrier, so the next setting's forward chain finds the planes free)
      adj_chain<NL - 1, CH, WL, false, LOGV>(x, y, re, im, tau, pc, nullptr);
      apply_phase<true, LOGV>(x, y, pos0, ym, off0);
#pragma unroll
      for (int i = 0; i < V; ++i) {
        ax[i] += x[i];
        ay[i] += y[i];
      }
    }
    // The slice's partial gradient (or the gradient itself when there is one slice).
    if (active) {
      float2* out = a.nA == 1 ? a.grad : a.P + (long long)slice * R * D;
      const rsrc_t ro = make_rsrc(out, (uint32_t)((long long)R * D * 8));
#pragma unroll
      for (int i = 0; i < V; ++i) bstore2(ax[i], ay[i], ro, vo0 + abase, off0(i) * 8u);
    }
    // Weight-gradient partial of atom r for this slice: tree over the vector's threads.
    red[tid] = h_acc;
    __syncthreads();
    for (int st = TA >> 1; st > 0; st >>= 1) {
      if (tau < st) red[tid] += red[tid + st];
      __syncthreads();
    }
    if (tau == 0 && active && a.part != nullptr) a.part[(long long)(1 + r) * a.nslots + slice] = red[tid];
    __syncthreads();
  }
}

// ------------------------------------------------------------------ fused slices (one-chunk states)
// States whose R atoms fit one work-group together (R 2^n <= 2^14): one pass per item =
// (instance, slice of settings) with every atom of a setting on chip at once, as in the fused
// low stage -- rotation, the atom sum alpha_r |phi_r|^2 through an LDS table, loss terms and
// g = dL/dp per outcome, the weight-gradient partial sums, alpha_r 2^-k g * phi through the
// adjoint rotation -- and the adjoint summed over the slice's settings in registers: one
// partial gradient per slice instead of one rotated vector per setting through HBM.
// Atom r is held by threads [r 2^(n-LOGV), (r+1) 2^(n-LOGV)); the launch is sized for the
// largest rank RM of its instances (threads of atoms beyond an instance's rank read zeros
// and write nothing).  ADJ = false: probabilities and loss only.
template <int NB, bool ADJ>
__global__ __launch_bounds__(512) void k_fs(const OcInst* __restrict__ tab, int k0, int k1, int total, int RM) {
  constexpr int LOGV = NB < 5 ? NB : 5;
  constexpr int V = 1 << LOGV;
  constexpr int U = 1 << NB;
  constexpr int UPAD = U + (U >> 5);
  constexpr int LOG_TA = NB - LOGV;
  constexpr int TA = 1 << LOG_TA;
  constexpr bool WL = LOG_TA <= 6;
  using CH = Chain<NB, LOGV>;
  constexpr int NL = CH::count();
  constexpr int LO0 = CH::lo(0);
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  const int atom = tid >> LOG_TA;
  const int tau = tid & (TA - 1);
  // LDS: wavefront-local transposes use one plane per atom, which also holds that atom's row
  // of the table alpha_r |phi_r|^2 (its threads write the row after their last transpose; the
  // other atoms read it only between the two barriers around the outcome loop); the g row
  // follows.  Work-group transposes use a real and an imaginary plane per atom; the table and
  // the g row alias the first rows (barriers separate the uses).
  float* planes = reinterpret_cast<float*>(smem);
  float* re = WL ? planes + (size_t)atom * UPAD : planes + (size_t)atom * 2 * UPAD;
  float* im = WL ? re : re + UPAD;
  float* qb = planes;
  float* gb = qb + (size_t)RM * UPAD;
  const size_t plane_rows = WL ? (size_t)RM + 1 : 2 * (size_t)RM;
  double* red = reinterpret_cast<double*>(smem + (((plane_rows * UPAD * 4) + 15) & ~(size_t)15));
  const uint32_t pos0 = (uint32_t)lay_pos<LOGV>(tau, 0, LO0);
  auto off0 = [](int i) { return (uint32_t)(i << LO0); };

  constexpr int NP = 4;  // data values per thread fetched ahead of the rotation
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
#pragma clang fp contract(off)
    const int k = oc_find(k0, k1, item, [&](int kk) { return tab[kk].itemA0; });
    const OcInst& a = tab[k];
    const int j = item - a.itemA0;
    const int s_beg = j * a.sA;
    const int s_end = min(a.B, s_beg + a.sA);
    const int R = a.R;
    const bool active = atom < R;
    const long long D = 1ll << NB;
    const float al = active ? (float)a.alpha[atom] : 0.0f;
    const float inv_b = (float)(1.0 / (double)a.B);
    const float eps_f = (float)a.eps;
    const uint32_t vo0 = pos0 * 8u;
    const bool gen = a.grad_p != nullptr;
    const bool row_data = gen || a.loss_kind != 2;
    const float* dsrc = gen ? a.grad_p : a.freqs;
    // the atom is read again for every setting (from L2); atoms beyond the rank read zeros
    const rsrc_t rs = make_rsrc(a.atoms, (uint32_t)((long long)R * D * 8));
    const uint32_t abase = (uint32_t)((long long)(active ? atom : R) * D * 8);
    float ax[V], ay[V];
#pragma unroll
    for (int i = 0; i < V; ++i) ax[i] = ay[i] = 0.0f;
    double loss_acc = 0.0, h_acc = 0.0;
    for (int b = s_beg; b < s_end; ++b) {
      const uint64_t pc = load_code(a.pc, b);
      const uint32_t ym = ymask_of(pc, NB);
      const float s2 = (float)ldexp(1.0, -nonz_count(pc, NB));
      const long long row = (long long)b * D;
      // this thread's outcomes are u = tid + jj * nthr; the first NP data values are fetched
      // before the rotation, so their loads overlap it, the rest in groups of NP
      float dv[NP];
#pragma unroll
      for (int jj = 0; jj < NP; ++jj) {
        const int u = tid + jj * nthr;
        dv[jj] = (row_data && u < U) ? dsrc[row + u] : 0.0f;
      }
      float x[V], y[V];
#pragma unroll
      for (int i = 0; i < V; ++i) bload2(x[i], y[i], rs, vo0 + abase, off0(i) * 8u);
      apply_phase<false, LOGV>(x, y, pos0, ym, off0);
      fwd_chain<0, CH, WL, false, LOGV>(x, y, re, im, tau, pc, nullptr);
      float* qrow = qb + (size_t)atom * UPAD + pad_base<LOGV, 0>(tau);
#pragma unroll
      for (int i = 0; i < V; ++i) qrow[pad_off<0>(i)] = al * fma(x[i], x[i], y[i] * y[i]);
      __syncthreads();
      for (int j0 = 0; tid + j0 * nthr < U; j0 += NP) {
        if (j0 > 0) {
#pragma unroll
          for (int jj = 0; jj < NP; ++jj) {
            const int u = tid + (j0 + jj) * nthr;
            dv[jj] = (row_data && u < U) ? dsrc[row + u] : 0.0f;
          }
        }
#pragma unroll
        for (int jj = 0; jj < NP; ++jj) {
        const int u = tid + (j0 + jj) * nthr;
        if (u >= U) continue;
        float pv = 0.0f;
        for (int r = 0; r < R; ++r) pv += qb[(size_t)r * UPAD + pad32(u)];
        pv *= s2;
        if (a.pbase != nullptr) pv += a.pbase[row + u];
        if (a.probs != nullptr) a.probs[row + u] = pv;
        float g = 0.0f;
        const float d = dv[jj];
        if (gen) {
          g = d;
        } else if (a.loss_kind == 0) {
          if (d > 0.0f) {
            const float fb = d * inv_b;
            const float piv = fmaf(pv, inv_b, eps_f);
            loss_acc -= (double)(fb * (__builtin_amdgcn_logf(piv) * 0.693147180559945309f));
            g = -(fb * inv_b) * __builtin_amdgcn_rcpf(piv);
          }
        } else if (a.loss_kind == 1) {
          const float rr = (pv - d) * inv_b;
          loss_acc += (double)(0.5f * rr * rr);
          g = rr * inv_b;
        }
        if (a.gneg != nullptr) a.gneg[row + u] = -g;
        if (ADJ) gb[pad32(u)] = g * s2;
        }
      }
      __syncthreads();
      if constexpr (ADJ) {
        float hl = 0.0f;
#pragma unroll
        for (int i = 0; i < V; ++i) {
          const float gv = gb[pad_base<LOGV, 0>(tau) + pad_off<0>(i)];
          hl = fma(gv, fma(x[i], x[i], y[i] * y[i]), hl);
          const float sc = al * gv;
          x[i] *= sc;
          y[i] *= sc;
        }
        h_acc += (double)hl;
        if constexpr (!WL) __syncthreads();  // every thread has read g before the planes are reused
        adj_chain<NL - 1, CH, WL, false, LOGV>(x, y, re, im, tau, pc, nullptr);
        apply_phase<true, LOGV>(x, y, pos0, ym, off0);
#pragma unroll
        for (int i = 0; i < V; ++i) {
          ax[i] += x[i];
          ay[i] += y[i];
        }
      }
      if constexpr (!WL) __syncthreads();  // the table and g rows alias the planes of the next setting
    }
    if constexpr (ADJ) {
      if (active) {
        float2* out = a.nA == 1 ? a.grad : a.P + (long long)j * R * D;
        const rsrc_t ro = make_rsrc(out, (uint32_t)((long long)R * D * 8));
#pragma unroll
        for (int i = 0; i < V; ++i) bstore2(ax[i], ay[i], ro, vo0 + abase, off0(i) * 8u);
      }
    }
    // Partials of this item (slot j): loss over the work-group, h_r over atom r's threads.
    if (a.part != nullptr) {
      if constexpr (ADJ) {
        red[tid] = h_acc;
        __syncthreads();
        for (int st = TA >> 1; st > 0; st >>= 1) {
          if (tau < st) red[tid] += red[tid + st];
          __syncthreads();
        }
        if (tau == 0 && active) a.part[(long long)(1 + atom) * a.nslots + j] = red[tid];
        __syncthreads();
      }
      red[tid] = loss_acc;
      __syncthreads();
      int np2 = 1;
      while (np2 < nthr) np2 <<= 1;
      for (int st = np2 >> 1; st > 0; st >>= 1) {
        if (tid < st && tid + st < nthr) red[tid] += red[tid + st];
        __syncthreads();
      }
      if (tid == 0) a.part[j] = red[0];
      __syncthreads();
    }
  }
}

// ------------------------------------------------------------------ slice sums, reductions, tangent
// grad[k][e] = sum over slices j of P[k][j][e] (instances with nA > 1).  A block takes 32
// consecutive elements; for each, eight threads sum the slices j = t, t + 8, ... in increasing
// order (independent loads, unrolled by four), and the eight sums are added in a fixed tree.
// Blocks [sumB0, sumB0 + ceil(R D / 32)) of the launch belong to instance k.
constexpr int kOcSumCols = 32;
constexpr int kOcSumThreads = 8;
__global__ __launch_bounds__(kOcSumCols * kOcSumThreads) void k_oc_sum(const OcInst* __restrict__ tab, int count) {
  __shared__ float2 part[kOcSumThreads][kOcSumCols];
  const int k = oc_find(0, count, (int)blockIdx.x, [&](int kk) { return tab[kk].sumB0; });
  const OcInst& a = tab[k];
  if (a.nA <= 1) return;
  const long long RD = (long long)a.R << a.n;
  const int col = threadIdx.x % kOcSumCols, t = threadIdx.x / kOcSumCols;
  const long long e = ((long long)blockIdx.x - a.sumB0) * kOcSumCols + col;
  float sx = 0.0f, sy = 0.0f;
  if (e < RD) {
    const float2* P = a.P + e;
    int jj = t;
    for (; jj + 3 * kOcSumThreads < a.nA; jj += 4 * kOcSumThreads) {
      const float2 v0 = P[(long long)jj * RD], v1 = P[(long long)(jj + kOcSumThreads) * RD];
      const float2 v2 = P[(long long)(jj + 2 * kOcSumThreads) * RD], v3 = P[(long long)(jj + 3 * kOcSumThreads) * RD];
      sx += v0.x;
      sy += v0.y;
      sx += v1.x;
      sy += v1.y;
      sx += v2.x;
      sy += v2.y;
      sx += v3.x;
      sy += v3.y;
    }
    for (; jj < a.nA; jj += kOcSumThreads) {
      const float2 v = P[(long long)jj * RD];
      sx += v.x;
      sy += v.y;
    }
  }
  part[t][col] = make_float2(sx, sy);
  __syncthreads();
  if (t == 0 && e < RD) {
    auto add = [](float2 u, float2 v) { return make_float2(u.x + v.x, u.y + v.y); };
    const float2 p01 = add(part[0][col], part[1][col]), p23 = add(part[2][col], part[3][col]);
    const float2 p45 = add(part[4][col], part[5][col]), p67 = add(part[6][col], part[7][col]);
    a.grad[e] = add(add(p01, p23), add(p45, p67));
  }
}

// Pauli codes of every instance's settings, one thread per setting: 2 bits per qubit, qubit j
// at index bit n-1-j (codes above 2 are taken as Z and raise bit 0 of the flag).  Blocks
// [decB0, decB0 + ceil(B / 256)) belong to instance k.
__global__ __launch_bounds__(256) void k_oc_decode(const OcInst* __restrict__ tab, int count, int* __restrict__ flag) {
  const int k = oc_find(0, count, (int)blockIdx.x, [&](int kk) { return tab[kk].decB0; });
  const OcInst& a = tab[k];
  const int b = ((int)blockIdx.x - a.decB0) * 256 + (int)threadIdx.x;
  if (b >= a.B) return;
  uint64_t v = 0;
  int bad = 0;
  for (int j = 0; j < a.n; ++j) {
    uint32_t c = a.settings[(size_t)b * a.n + j];
    if (c > 2u) {
      bad = 1;
      c = 2u;
    }
    v |= (uint64_t)c << (2 * (a.n - 1 - j));
  }
  a.pc_out[b] = v;
  if (bad) atomicOr(flag, 1);
}

hipError_t launch_oc_decode(const OcInst* tab, int count, int blocks, int* flag, hipStream_t st) {
  if (blocks > 0) k_oc_decode<<<blocks, 256, 0, st>>>(tab, count, flag);
  return hipGetLastError();
}

__device__ __forceinline__ double oc_block_sum(double v, double* red) {
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

// Work-group (k, row): row 0 sums the loss slots, row 1 + r the weight-gradient slots of atom r.
__global__ __launch_bounds__(256) void k_oc_rowsum(const OcInst* __restrict__ tab) {
  __shared__ double red[256];
  const OcInst& a = tab[blockIdx.x];
  const int row = blockIdx.y;
  if (row > a.R || a.part == nullptr) return;
  if (row == 0 && a.loss == nullptr) return;
  if (row > 0 && a.wgrad == nullptr) return;
  double acc = 0.0;
  for (long long i = threadIdx.x; i < a.nslots; i += 256) acc += a.part[(long long)row * a.nslots + i];
  const double r = oc_block_sum(acc, red);
  if (threadIdx.x == 0) {
    if (row == 0)
      *a.loss = r;
    else
      a.wgrad[row - 1] = r;
  }
}

// Work-group (k, r): grad_r -= psi_r <psi_r, grad_r> with the inner product in FP64.
// One work-group of 1024 threads per (instance, atom): the vector is at most 2^14 long, so
// each thread takes at most 16 elements per pass; the dot product is summed over each
// wavefront by a fixed butterfly of lane exchanges, then over the wavefronts in order.
__global__ __launch_bounds__(1024) void k_oc_tangent(const OcInst* __restrict__ tab) {
  __shared__ double red[2][16];
  const OcInst& a = tab[blockIdx.x];
  const int r = blockIdx.y;
  if (!a.tangent || r >= a.R) return;
  const long long D = 1ll << a.n;
  const float2* psi = reinterpret_cast<const float2*>(a.atoms) + (long long)r * D;
  float2* grad = a.grad + (long long)r * D;
  double sre = 0.0, sim = 0.0;
  for (long long i = threadIdx.x; i < D; i += 1024) {
    const float2 p = psi[i], g = grad[i];
    sre += (double)p.x * g.x + (double)p.y * g.y;  // conj(p) g
    sim += (double)p.x * g.y - (double)p.y * g.x;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    sre += __shfl_xor(sre, o);
    sim += __shfl_xor(sim, o);
  }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][wave] = sre;
    red[1][wave] = sim;
  }
  __syncthreads();
  double tr = 0.0, ti = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
    tr += red[0][w];
    ti += red[1][w];
  }
  const float dr = (float)tr;
  const float di = (float)ti;
  for (long long i = threadIdx.x; i < D; i += 1024) {
    const float2 p = psi[i];
    float2 g = grad[i];
    g.x -= p.x * dr - p.y * di;
    g.y -= p.x * di + p.y * dr;
    grad[i] = g;
  }
}

// The instance table is written on the device from by-value chunks, so a captured graph
// holds it in its kernel parameters.
__global__ void k_oc_stage(const OcChunk c, OcInst* __restrict__ tab) {
  const int words = c.count * (int)(sizeof(OcInst) / 4);
  const uint32_t* src = reinterpret_cast<const uint32_t*>(c.a);
  uint32_t* dst = reinterpret_cast<uint32_t*>(tab + c.first);
  for (int w = threadIdx.x; w < words; w += blockDim.x) dst[w] = src[w];
}

// ------------------------------------------------------------------ launchers
size_t oc_lds_bytes(int n, int logv) {
  const int LOG_TA = n - logv;
  const int TA = 1 << LOG_TA;
  const int NT = TA > 256 ? TA : 256;
  const size_t U = (size_t)1 << n;
  const size_t planes = (size_t)(NT / TA) * (LOG_TA <= 6 ? 1 : 2) * (U + (U >> 5)) * 4;
  return ((planes + 15) & ~(size_t)15) + (size_t)NT * sizeof(double);
}

int oc_threads_of(int n, int logv) { return (1 << (n - logv)) > 256 ? (1 << (n - logv)) : 256; }

template <int NB, int LOGV>
static const void* oc_fn(bool adj) {
  return adj ? reinterpret_cast<const void*>(&k_oc_adj<NB, LOGV>) : reinterpret_cast<const void*>(&k_oc_fwd<NB, LOGV>);
}

template <int NB, int LOGV>
static hipError_t oc_launch(bool adj, const OcInst* tab, int k0, int k1, int total, int grid, hipStream_t st) {
  const size_t lds = oc_lds_bytes(NB, LOGV);
  const hipError_t e = hipFuncSetAttribute(oc_fn<NB, LOGV>(adj), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (adj)
    k_oc_adj<NB, LOGV><<<grid, oc_threads<NB, LOGV>(), lds, st>>>(tab, k0, k1, total);
  else
    k_oc_fwd<NB, LOGV><<<grid, oc_threads<NB, LOGV>(), lds, st>>>(tab, k0, k1, total);
  return hipGetLastError();
}

template <int NB, int LOGV>
static int oc_occ(bool adj) {
  const size_t lds = oc_lds_bytes(NB, LOGV);
  if (hipFuncSetAttribute(oc_fn<NB, LOGV>(adj), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return 1;
  int blocks = 0;
  const hipError_t e =
      adj ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_oc_adj<NB, LOGV>, oc_threads<NB, LOGV>(), lds)
          : hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_oc_fwd<NB, LOGV>, oc_threads<NB, LOGV>(), lds);
  return (e == hipSuccess && blocks > 0) ? blocks : 1;
}

// Supported (n, values per thread): 2^5 for n = 11..14, 2^4 for n = 13, 14 (twice the threads).
bool oc_shape_ok(int n, int logv) { return (n >= 11 && n <= 14 && logv == 5) || ((n == 13 || n == 14) && logv == 4); }

hipError_t launch_oc_pass(int n, int logv, bool adj, const OcInst* tab, int k0, int k1, int total, int grid,
                          hipStream_t st) {
  if (logv == 4) {
    if (n == 13) return oc_launch<13, 4>(adj, tab, k0, k1, total, grid, st);
    if (n == 14) return oc_launch<14, 4>(adj, tab, k0, k1, total, grid, st);
    return hipErrorInvalidValue;
  }
  switch (n) {
    case 11: return oc_launch<11, 5>(adj, tab, k0, k1, total, grid, st);
    case 12: return oc_launch<12, 5>(adj, tab, k0, k1, total, grid, st);
    case 13: return oc_launch<13, 5>(adj, tab, k0, k1, total, grid, st);
    case 14: return oc_launch<14, 5>(adj, tab, k0, k1, total, grid, st);
  }
  return hipErrorInvalidValue;
}

int oc_blocks_per_cu(int n, int logv, bool adj) {
  if (logv == 4) {
    if (n == 13) return oc_occ<13, 4>(adj);
    if (n == 14) return oc_occ<14, 4>(adj);
    return 1;
  }
  switch (n) {
    case 11: return oc_occ<11, 5>(adj);
    case 12: return oc_occ<12, 5>(adj);
    case 13: return oc_occ<13, 5>(adj);
    case 14: return oc_occ<14, 5>(adj);
  }
  return 1;
}

size_t fs_lds_bytes(int n, int RM) {
  const int logv = n < 5 ? n : 5;
  const bool wl = n - logv <= 6;
  const size_t U = (size_t)1 << n;
  const size_t rows = wl ? (size_t)RM + 1 : 2 * (size_t)RM;
  const size_t nthr = (size_t)RM << (n - logv);
  return ((rows * (U + (U >> 5)) * 4 + 15) & ~(size_t)15) + nthr * sizeof(double);
}

int fs_threads(int n, int RM) { return RM << (n - (n < 5 ? n : 5)); }

template <int NB>
static hipError_t fs_launch(bool adj, const OcInst* tab, int k0, int k1, int total, int RM, int grid, hipStream_t st) {
  const size_t lds = fs_lds_bytes(NB, RM);
  const void* fn = adj ? reinterpret_cast<const void*>(&k_fs<NB, true>) : reinterpret_cast<const void*>(&k_fs<NB, false>);
  const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (adj)
    k_fs<NB, true><<<grid, fs_threads(NB, RM), lds, st>>>(tab, k0, k1, total, RM);
  else
    k_fs<NB, false><<<grid, fs_threads(NB, RM), lds, st>>>(tab, k0, k1, total, RM);
  return hipGetLastError();
}

template <int NB>
static int fs_occ(bool adj, int RM) {
  const size_t lds = fs_lds_bytes(NB, RM);
  const void* fn = adj ? reinterpret_cast<const void*>(&k_fs<NB, true>) : reinterpret_cast<const void*>(&k_fs<NB, false>);
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) return 1;
  int blocks = 0;
  const hipError_t e = adj ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_fs<NB, true>, fs_threads(NB, RM), lds)
                           : hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_fs<NB, false>, fs_threads(NB, RM), lds);
  return (e == hipSuccess && blocks > 0) ? blocks : 1;
}

#define QST_FS_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14)

hipError_t launch_fs_pass(int n, bool adj, const OcInst* tab, int k0, int k1, int total, int RM, int grid,
                          hipStream_t st) {
  if (((long long)RM << n) > 16384) return hipErrorInvalidValue;
  switch (n) {
#define QST_C(N) \
  case N: return fs_launch<N>(adj, tab, k0, k1, total, RM, grid, st);
    QST_FS_CASES(QST_C)
#undef QST_C
  }
  return hipErrorInvalidValue;
}

int fs_blocks_per_cu(int n, bool adj, int RM) {
  switch (n) {
#define QST_C(N) \
  case N: return fs_occ<N>(adj, RM);
    QST_FS_CASES(QST_C)
#undef QST_C
  }
  return 1;
}

hipError_t launch_oc_stage(const OcChunk& c, OcInst* tab, hipStream_t st) {
  k_oc_stage<<<1, 256, 0, st>>>(c, tab);
  return hipGetLastError();
}

hipError_t launch_oc_finish(const OcInst* tab, int count, int sum_blocks, int rmax, bool rows, bool tangent,
                            hipStream_t st) {
  if (sum_blocks > 0) k_oc_sum<<<sum_blocks, kOcSumCols * kOcSumThreads, 0, st>>>(tab, count);
  if (rows) k_oc_rowsum<<<dim3(count, rmax + 1), 256, 0, st>>>(tab);
  if (tangent) k_oc_tangent<<<dim3(count, rmax), 1024, 0, st>>>(tab);
  return hipGetLastError();
}

}  // namespace qst
