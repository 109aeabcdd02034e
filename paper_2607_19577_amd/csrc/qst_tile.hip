// One HBM pass per group of four qubits: the 16x16 complex Kronecker tile of a
// setting, V_g = V_{c3} (x) V_{c2} (x) V_{c1} (x) V_{c0} over index bits
// [gb, gb+4), applied to every (setting, atom) vector on the matrix cores.
//
// Tiles use the unnormalised rotations (X: [[1,1],[1,-1]], Y: [[1,-i],[1,i]],
// Z: identity), whose entries 0, +-1, +-i are exact in FP16 and BF16; the scale
// 2^-k_b is applied on |phi|^2 by the pointwise step, as on the other paths.
// A complex product U B is four real 16x16x16 MFMAs (FP32 accumulation):
//   Re = Ur Br - Ui Bi,   Im = Ur Bi + Ui Br.
// FP16 operands: each 16x16 block is scaled by a power of two so that its
// largest entry is near 2^14 before rounding (the sensitivities of the adjoint
// are far below FP16's normal range otherwise), and unscaled after the MFMA.
// BF16 operands: each amplitude is split into a high and a low BF16 part
// (x = hi + lo + O(2^-16 x)), so the pass keeps about 16 significant bits.
//
// Operand layouts of v_mfma_f32_16x16x16 (checked on the device): lane l holds
// A[l%16][4(l/16)+v], B[4(l/16)+v][l%16] and C[4(l/16)+v][l%16], v = 0..3, so a
// lane reads and writes the same four amplitudes (B row k <-> C row i).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qst_internal.hpp"

namespace qst {

namespace {

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

// Entry (a, b) of the unnormalised single-qubit rotation for code c, as a power of i
// (0..3), or -1 for zero.  Forward: X: (-1)^{ab} = i^{2ab}; Y: 1, -i / 1, i; Z: delta_ab.
__device__ __forceinline__ int rot_pow(uint32_t c, int a, int b) {
  if (c == 0u) return 2 * (a & b);
  if (c == 1u) return b ? (a ? 1 : 3) : 0;
  return a == b ? 0 : -1;
}

// Tile entry U[i][k] (forward) or (U^dagger)[i][k] = conj(U[k][i]) (adjoint) as (re, im).
template <bool ADJ>
__device__ __forceinline__ void tile_entry(uint32_t codes4, int i, int k, float& re, float& im) {
  int m = 0;
  for (int q = 0; q < 4; ++q) {
    const uint32_t c = (codes4 >> (2 * q)) & 3u;
    const int a = ADJ ? (k >> q) & 1 : (i >> q) & 1;
    const int b = ADJ ? (i >> q) & 1 : (k >> q) & 1;
    const int p = rot_pow(c, a, b);
    if (p < 0) {
      re = 0.f;
      im = 0.f;
      return;
    }
    m += p;
  }
  if (ADJ) m = -m;
  m &= 3;
  re = m == 0 ? 1.f : (m == 2 ? -1.f : 0.f);
  im = m == 1 ? 1.f : (m == 3 ? -1.f : 0.f);
}

__device__ __forceinline__ short bf16_rn(float x) {
  const uint32_t u = __float_as_uint(x);
  const uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);  // round to nearest even (finite inputs)
  return (short)(r >> 16);
}
__device__ __forceinline__ float bf16_val(short h) { return __uint_as_float((uint32_t)(uint16_t)h << 16); }

template <int MODE, bool ADJ>  // MODE 0: FP16 operands, 1: BF16 high/low operands
__global__ __launch_bounds__(256) void k_tile_pass(float2* __restrict__ X, int S, int R, long long D, int gb,
                                                   const uint64_t* __restrict__ pc, int b0) {
  const int lane = threadIdx.x & 63;
  const int col = lane & 15;
  const int kq = 4 * (lane >> 4);
  const long long nblk = D >> 8;  // blocks of 16 columns x 16 group values
  const long long items = (long long)S * R * nblk;
  const long long wave = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const long long nwaves = (long long)gridDim.x * (blockDim.x >> 6);
  const long long lowmask = (1ll << gb) - 1;
  int cur_s = -1;
  float4_t ur = {0, 0, 0, 0}, ui = {0, 0, 0, 0};
  for (long long it = wave; it < items; it += nwaves) {
    const int s = (int)(it / ((long long)R * nblk));
    const long long rem = it - (long long)s * R * nblk;
    const long long vec = (long long)s * R + rem / nblk;
    const long long blk = rem % nblk;
    if (s != cur_s) {
      cur_s = s;
      const uint32_t codes4 = (uint32_t)((pc[b0 + s] >> (2 * gb)) & 0xffull);
      for (int v = 0; v < 4; ++v) {
        float re, im;
        tile_entry<ADJ>(codes4, col, kq + v, re, im);  // A[row = lane%16][k = 4(lane/16)+v]
        ur[v] = re;
        ui[v] = im;
      }
    }
    // the 16 columns of this block, group value k inserted at bits [gb, gb+4)
    const long long c = blk * 16 + col;
    const long long base = vec * D + (((c & ~lowmask) << 4) | (c & lowmask));
    float2 x[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) x[v] = X[base + ((long long)(kq + v) << gb)];
    float4_t cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
    if constexpr (MODE == 0) {
      float m = 0.f;
#pragma unroll
      for (int v = 0; v < 4; ++v) m = fmaxf(m, fmaxf(fabsf(x[v].x), fabsf(x[v].y)));
      for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
      int e = 0;
      if (m > 0.f) (void)frexpf(m, &e);
      const float up = ldexpf(1.f, 14 - e), down = ldexpf(1.f, e - 14);
      half4_t ar, ai, an, br, bi;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        ar[v] = (_Float16)ur[v];
        ai[v] = (_Float16)ui[v];
        an[v] = (_Float16)(-ui[v]);
        br[v] = (_Float16)(x[v].x * up);
        bi[v] = (_Float16)(x[v].y * up);
      }
      cr = __builtin_amdgcn_mfma_f32_16x16x16f16(ar, br, cr, 0, 0, 0);
      cr = __builtin_amdgcn_mfma_f32_16x16x16f16(an, bi, cr, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f32_16x16x16f16(ar, bi, ci, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f32_16x16x16f16(ai, br, ci, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        cr[v] *= down;
        ci[v] *= down;
      }
    } else {
      bf16x4_t ar, ai, an, rh, rl, ih, il;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        ar[v] = bf16_rn(ur[v]);
        ai[v] = bf16_rn(ui[v]);
        an[v] = bf16_rn(-ui[v]);
        rh[v] = bf16_rn(x[v].x);
        rl[v] = bf16_rn(x[v].x - bf16_val(rh[v]));
        ih[v] = bf16_rn(x[v].y);
        il[v] = bf16_rn(x[v].y - bf16_val(ih[v]));
      }
      cr = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ar, rl, cr, 0, 0, 0);
      cr = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(an, il, cr, 0, 0, 0);
      cr = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ar, rh, cr, 0, 0, 0);
      cr = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(an, ih, cr, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ar, il, ci, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ai, rl, ci, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ar, ih, ci, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ai, rh, ci, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) X[base + ((long long)(kq + v) << gb)] = float2{cr[v], ci[v]};
  }
}

}  // namespace

hipError_t launch_tile_pass(void* X, int S, int R, long long D, int gb, const uint64_t* pc, int b0, bool adj,
                            bool bf16, hipStream_t st) {
  if (D < 256 || gb < 0 || (1ll << (gb + 4)) > D) return hipErrorInvalidValue;
  const long long items = (long long)S * R * (D >> 8);
  long long nb = (items + 3) / 4;  // four waves per work-group
  if (nb > 16384) nb = 16384;
  float2* x = reinterpret_cast<float2*>(X);
  if (!bf16 && !adj) k_tile_pass<0, false><<<(unsigned)nb, 256, 0, st>>>(x, S, R, D, gb, pc, b0);
  if (!bf16 && adj) k_tile_pass<0, true><<<(unsigned)nb, 256, 0, st>>>(x, S, R, D, gb, pc, b0);
  if (bf16 && !adj) k_tile_pass<1, false><<<(unsigned)nb, 256, 0, st>>>(x, S, R, D, gb, pc, b0);
  if (bf16 && adj) k_tile_pass<1, true><<<(unsigned)nb, 256, 0, st>>>(x, S, R, D, gb, pc, b0);
  return hipGetLastError();
}

}  // namespace qst
