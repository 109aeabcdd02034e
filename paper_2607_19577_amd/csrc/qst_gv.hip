// G v products of the spectral slot (eqs. density-product, negative-gradient-product) for
// states with high bits: one vector v (R = 1), Pauli settings, FP32,
//   G v = sum_b V_b^dagger diag(alpha 2^-k_b g_b) V_b v.
//
// V_b factors into H_b, the rotations of the qubits on the high index bits [n_lo, n), and L_b,
// those on the low bits [0, n_lo) with their Y phases; the two act on different bits and
// commute.  Settings whose high codes are equal (a pattern P) share H_b, so
//   G v = sum_P H_P^dagger [ sum_{b in P} L_b^dagger diag(alpha 2^-k_b g_b) L_b ] H_P v.
// Stage A forms X_P = H_P v once per pattern (codes of the low qubits set to Z, so it applies
// only the high phases), this kernel forms W_P = [ ... ] X_P chunk by chunk, and stage C sums
// H_P^dagger W_P over the patterns.  With n_lo = 14 there are at most 3^(n-14) <= 729 patterns,
// so X and W cross HBM once per pattern rather than once per setting: at n = 20 and 2000
// random settings about 680 patterns, 2.9 times fewer bytes of X and W.
//
// Item = (pattern, high index h): the 2^14-amplitude chunk h of X_P stays in registers while
// each member's low phase, low butterflies, sensitivity scale, adjoint butterflies and
// conjugate phase run on a copy, summed in registers; one store of W_P's chunk per item.
#include "qst_stages.hpp"

namespace qst {

namespace {

__device__ __forceinline__ int load_int(const int* p, int i) {
  using ci32ptr = const __attribute__((address_space(4))) int*;
  return ((ci32ptr)(p))[__builtin_amdgcn_readfirstlane(i)];
}

__device__ __forceinline__ float4 ld_g4(const float* p) { return *reinterpret_cast<const float4*>(p); }

}  // namespace

template <int LOGV>
__global__ __launch_bounds__(1 << (kGvLoBits - LOGV)) void k_gv_lo(const GvArgs a) {
  constexpr int NB = kGvLoBits;
  constexpr int V = 1 << LOGV;
  constexpr int U = 1 << NB;
  constexpr int UPAD = U + (U >> 5);
  using CH = Chain<NB, LOGV>;
  constexpr int NL = CH::count();
  constexpr int LO0 = CH::lo(0);
  extern __shared__ __align__(16) unsigned char smem[];
  const int tau = threadIdx.x;
  float* re = reinterpret_cast<float*>(smem);
  float* im = re + UPAD;
  const uint32_t pos0 = (uint32_t)lay_pos<LOGV>(tau, 0, LO0);
  const uint32_t vo0 = pos0 * 8u;
  auto off0 = [](int i) { return (uint32_t)(i << LO0); };
  const int nh = a.n - NB;
  const long long D = 1ll << a.n;
  const int total = a.S << nh;
  const float al = (float)a.alpha[0];

  for (int item = blockIdx.x; item < total; item += gridDim.x) {
#pragma clang fp contract(off)
    const int sp = item >> nh;
    const int hh = item & ((1 << nh) - 1);
    const long long cb = (long long)sp * D + ((long long)hh << NB);
    const rsrc_t rx = make_rsrc(a.X + cb, (uint32_t)U * 8u);
    float xs[V], ys[V], ax[V], ay[V];
#pragma unroll
    for (int i = 0; i < V; ++i) {
      bload2(xs[i], ys[i], rx, vo0, off0(i) * 8u);
      ax[i] = ay[i] = 0.0f;
    }
    const int m0 = load_int(a.goff, a.p0 + sp), m1 = load_int(a.goff, a.p0 + sp + 1);
    for (int m = m0; m < m1; ++m) {
      const int b = load_int(a.perm, m);
      const uint64_t pc = load_code(a.pc, b);
      const uint32_t ym = ymask_of(pc, NB) & (uint32_t)(U - 1);  // the low bits' Y qubits
      const float s2 = al * (float)ldexp(1.0, -nonz_count(pc, a.n));
      float x[V], y[V];
#pragma unroll
      for (int i = 0; i < V; ++i) x[i] = xs[i], y[i] = ys[i];
      apply_phase<false, LOGV>(x, y, pos0, ym, off0);
      fwd_chain<0, CH, false, false, LOGV, false>(x, y, re, im, tau, pc, nullptr);
      // this thread's outcomes of the chunk (final layout lo = 0)
      const float* gr = a.g + (long long)b * D + ((long long)hh << NB) + ((long long)tau << LOGV);
#pragma unroll
      for (int q = 0; q < V / 4; ++q) {
        const float4 v = ld_g4(gr + 4 * q);
        const float c0 = s2 * v.x, c1 = s2 * v.y, c2 = s2 * v.z, c3 = s2 * v.w;
        x[4 * q] *= c0, y[4 * q] *= c0;
        x[4 * q + 1] *= c1, y[4 * q + 1] *= c1;
        x[4 * q + 2] *= c2, y[4 * q + 2] *= c2;
        x[4 * q + 3] *= c3, y[4 * q + 3] *= c3;
      }
      adj_chain<NL - 1, CH, false, false, LOGV>(x, y, re, im, tau, pc, nullptr);
      apply_phase<true, LOGV>(x, y, pos0, ym, off0);
#pragma unroll
      for (int i = 0; i < V; ++i) {
        ax[i] += x[i];
        ay[i] += y[i];
      }
    }
    const rsrc_t rw = make_rsrc(a.W + cb, (uint32_t)U * 8u);
#pragma unroll
    for (int i = 0; i < V; ++i) bstore2(ax[i], ay[i], rw, vo0, off0(i) * 8u);
  }
}

size_t gv_lds_bytes() {
  constexpr size_t U = (size_t)1 << kGvLoBits;
  return 2 * (U + (U >> 5)) * 4;
}

template <int LOGV>
static int gv_occ() {
  const size_t lds = gv_lds_bytes();
  if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gv_lo<LOGV>), hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lds) != hipSuccess)
    return 1;
  int blocks = 0;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_gv_lo<LOGV>, 1 << (kGvLoBits - LOGV), lds);
  return (e == hipSuccess && blocks > 0) ? blocks : 1;
}

int gv_blocks_per_cu(int logv) { return logv == 5 ? gv_occ<5>() : 1; }

template <int LOGV>
static hipError_t gv_launch(const GvArgs& a, int grid, hipStream_t st) {
  const size_t lds = gv_lds_bytes();
  const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gv_lo<LOGV>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  k_gv_lo<LOGV><<<grid, 1 << (kGvLoBits - LOGV), lds, st>>>(a);
  return hipGetLastError();
}

hipError_t launch_gv_lo(const GvArgs& a, int logv, int grid, hipStream_t st) {
  if (a.n <= kGvLoBits || a.n > 20 || a.S < 1 || grid < 1) return hipErrorInvalidValue;
  if (logv == 5) return gv_launch<5>(a, grid, st);
  return hipErrorInvalidValue;
}

}  // namespace qst
