// Device helpers shared by the butterfly kernels: complex types, the unscaled
// single-qubit Pauli rotations, in-register butterflies, layouts and the
// padded LDS indexing used by the transposes.
//
// A "block" is a power-of-two set of amplitudes a work-group holds on chip.
// Each thread keeps V = 2^LOGV of them in registers.  A *layout* is named by
// `lo`: the thread's in-register index i supplies block bits [lo, lo+LOGV)
// and the thread index supplies the remaining bits in increasing order, so
// consecutive threads touch consecutive addresses whenever lo > 0 (coalesced
// global access).  A qubit whose bit lies in [lo, lo+LOGV) is a butterfly
// between two registers of one thread; moving between layouts is a transpose
// through LDS.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qst {

template <typename T> struct cx_of;
template <> struct cx_of<float> { using type = float2; };
template <> struct cx_of<double> { using type = double2; };
template <typename T> using cx = typename cx_of<T>::type;

// Pauli codes as stored in a setting: X = 0, Y = 1, Z = 2.  Codes 2 and 3 mean
// "no rotation" inside the 2-bit code words handed to xform_xz().
constexpr uint32_t CODE_SKIP = 2u;

// LDS index with one pad slot every 32 elements: a stride-32 access pattern
// (in-register bits at the bottom of the block) then spreads over all banks.
__device__ __forceinline__ int pad32(int p) { return p + (p >> 5); }

// Block position of register i of thread tau in the layout `lo`.
template <int LOGV>
__device__ __forceinline__ int lay_pos(int tau, int i, int lo) {
  const int m = (1 << lo) - 1;
  return ((tau & ~m) << LOGV) | (i << lo) | (tau & m);
}

// pad32(lay_pos(tau, i, lo)) split into a per-thread base and a per-register
// constant: with p = H | (i << lo) | L (H a multiple of 2^(lo+LOGV), L < 2^lo),
// p >> 5 = H >> 5 + (lo >= 5 ? (i << (lo-5)) + (L >> 5) : i >> (5-lo)), so
// the register part becomes an immediate LDS offset.
template <int LOGV, int LO>
__device__ __forceinline__ int pad_base(int tau) {
  constexpr int m = (1 << LO) - 1;
  const int H = (tau & ~m) << LOGV;
  const int L = tau & m;
  return H + L + (H >> 5) + (LO >= 5 ? (L >> 5) : 0);
}
template <int LO>
__host__ __device__ constexpr int pad_off(int i) {
  return (i << LO) + (LO >= 5 ? (i << (LO - 5)) : (i >> (5 - LO)));
}

// Unscaled rotations: sqrt2 * V_X = [[1,1],[1,-1]], sqrt2 * V_Y = [[1,-i],[1,i]]
// (rows <+| and <-|, resp. <+i| and <-i|); the pair is (a, b) = (bit 0, bit 1).
// The 1/sqrt2 factors are applied once per setting as the exact power of two
// 2^(-k_b) on |phi|^2.
//
// These exact rotations serve the single-pass kernels: b' is formed first and
// a' is then recovered as 2a - b' with one fused multiply-add (a' = a + s,
// b' = a - s); the extra rounding is one ulp of |(a, b)|.
template <typename T>
__device__ __forceinline__ void bf_x(T& ax, T& ay, T& bx, T& by) {
  bx = ax - bx;
  by = ay - by;
  ax = fma(T(2), ax, -bx);
  ay = fma(T(2), ay, -by);
}
// a' = a - i b, b' = a + i b
template <typename T>
__device__ __forceinline__ void bf_y(T& ax, T& ay, T& bx, T& by) {
  const T nbx = ax - by;
  by = ay + bx;
  bx = nbx;
  ax = fma(T(2), ax, -bx);
  ay = fma(T(2), ay, -by);
}
// Adjoint of the Y rotation, [[1,1],[i,-i]]: a' = a + b, b' = i (a - b)
template <typename T>
__device__ __forceinline__ void bf_yh(T& ax, T& ay, T& bx, T& by) {
  const T nbx = by - ay;
  by = ax - bx;
  bx = nbx;
  ax = fma(T(2), ax, -by);
  ay = fma(T(2), ay, bx);
}
// Complex-pair forms (used by the single-pass reference kernels).
template <typename C2> __device__ __forceinline__ void bf_x(C2& a, C2& b) { bf_x(a.x, a.y, b.x, b.y); }
template <typename C2> __device__ __forceinline__ void bf_y(C2& a, C2& b) { bf_y(a.x, a.y, b.x, b.y); }
template <typename C2> __device__ __forceinline__ void bf_yh(C2& a, C2& b) { bf_yh(a.x, a.y, b.x, b.y); }

// Phase-split form (used by the staged kernels).  V_Y = H diag(1, -i) with the
// diagonal on the input side, and diagonals on different qubits commute with
// everything else, so for a setting with Y-qubit mask ymask
//     V_b = (x)_k M_k  *  diag((-i)^popcount(v & ymask)),
// M_k = H for X and Y bits and the identity for Z bits.  The kernels apply the
// per-element phase once per setting where the state enters the rotation
// (forward) or leaves it (adjoint: the conjugate phase after the M's); every
// X or Y bit in between is the same in-place butterfly a' = a + b,
// b' = a' - 2b (H is its own adjoint; the extra rounding is one ulp of
// |(a, b)|), and a Z bit is a uniform branch around it.
template <int K, int LOGV, typename T>
__device__ __forceinline__ void bit_xz(T (&x)[1 << LOGV], T (&y)[1 << LOGV], uint32_t c) {
  if (c >= 2u) return;
#pragma unroll
  for (int i = 0; i < (1 << LOGV); ++i) {
    if (i & (1 << K)) continue;
    const int j = i | (1 << K);
    x[i] = x[i] + x[j];
    y[i] = y[i] + y[j];
    x[j] = fma(T(-2), x[j], x[i]);
    y[j] = fma(T(-2), y[j], y[i]);
  }
}

template <int K, int LOGV, uint32_t ACTIVE, typename T>
__device__ __forceinline__ void xform_xz_bit(T (&x)[1 << LOGV], T (&y)[1 << LOGV], uint32_t codes) {
  if constexpr (K < LOGV) {
    if constexpr ((ACTIVE >> K) & 1u) bit_xz<K, LOGV>(x, y, (codes >> (2 * K)) & 3u);
    xform_xz_bit<K + 1, LOGV, ACTIVE>(x, y, codes);
  }
}

template <int LOGV, uint32_t ACTIVE, typename T>
__device__ __forceinline__ void xform_xz(T (&x)[1 << LOGV], T (&y)[1 << LOGV], uint32_t codes) {
  xform_xz_bit<0, LOGV, ACTIVE>(x, y, codes);
}

// The per-setting coefficients of general settings are read through the constant address
// space: their addresses are uniform, so the loads become scalar loads into SGPRs (issued
// early and batched) instead of one vector load and wait per coefficient.
using cfptr = const __attribute__((address_space(4))) float*;
__device__ __forceinline__ cfptr to_const(const float* p) { return (cfptr)(p); }

// A value that is the same in every lane, moved to a scalar register (a uniform branch
// on it then needs no lane mask).
__device__ __forceinline__ float uniform_f32(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// General local settings in rotation form.  The decode writes each qubit's matrix as
// P R diag(1, e): the outcome-side phases P drop out of |phi|^2 and of V^dagger diag(g) V,
// the input-side phases diag(1, e) of all qubits commute with every rotation and are
// applied once per element (apply_gphase), and what is left per qubit is the real
// rotation R = [[c, -s], [s, c]] (adjoint: its transpose, the angle negated).  It is
// applied as three shears (lifting): a -= t b, b += s a, a -= t b with t = tan(theta/2)
// and s = sin(theta), theta in [0, pi/2], stored at um + 8 q as (t, s) for index bit q
// (uniform across the work-group): six multiply-adds per pair, in place, and exact up to
// one rounding per shear.  The identity (t = s = 0) runs the same code: a branch around
// it makes the compiler keep both versions of the registers live at the join and spill.
template <int K, int LOGV, bool ADJ, uint32_t ACTIVE, typename T>
__device__ __forceinline__ void xform_gen_bit(T (&x)[1 << LOGV], T (&y)[1 << LOGV], cfptr um, int qidx0) {
  if constexpr (K < LOGV) {
    if constexpr ((ACTIVE >> K) & 1u) {
      const cfptr m = um + 8 * (qidx0 + K);
      const T tv = uniform_f32(m[0]), sv = uniform_f32(m[1]);
      const T nt = ADJ ? tv : -tv;  // -t of the applied angle
      const T s = ADJ ? -sv : sv;
#pragma unroll
      for (int i = 0; i < (1 << LOGV); ++i) {
        if (i & (1 << K)) continue;
        const int j = i | (1 << K);
        x[i] = fma(nt, x[j], x[i]);
        y[i] = fma(nt, y[j], y[i]);
        x[j] = fma(s, x[i], x[j]);
        y[j] = fma(s, y[i], y[j]);
        x[i] = fma(nt, x[j], x[i]);
        y[i] = fma(nt, y[j], y[i]);
      }
    }
    xform_gen_bit<K + 1, LOGV, ADJ, ACTIVE>(x, y, um, qidx0);
  }
}

template <int LOGV, bool ADJ, uint32_t ACTIVE, typename T>
__device__ __forceinline__ void xform_gen(T (&x)[1 << LOGV], T (&y)[1 << LOGV], cfptr um, int qidx0) {
  xform_gen_bit<0, LOGV, ADJ, ACTIVE>(x, y, um, qidx0);
}

// The input-side phase of general settings: element v gets prod_q e_q^(bit q of v), e_q the
// phase of index bit q of an n-bit index, given by eq(q) as (re, im) (uniform); CONJ
// multiplies by its conjugate (the adjoint, after the rotations).  Register i holds index
// base | off(i), where off maps register bits to distinct index bits outside base's.  The
// phase of base is a product over its set bits; the register part comes from two tables
// (register bits 0..2 and 3..4) built by doubling, so no phase is more than six products deep.
template <bool CONJ, int LOGV, typename T, typename Off, typename Eq>
__device__ __forceinline__ void apply_gphase(T (&x)[1 << LOGV], T (&y)[1 << LOGV], uint32_t base, int n, Off off,
                                             Eq eq) {
  constexpr int V = 1 << LOGV;
  constexpr int LA = LOGV < 3 ? LOGV : 3;  // register bits of the first table
  constexpr int NA = 1 << LA, NB = V >> LA;
  T br = T(1), bi = T(0);
  for (int q = 0; q < n; ++q) {
    const float2 e = eq(q);
    const T nr = fma(br, (T)e.x, -bi * (T)e.y), ni = fma(br, (T)e.y, bi * (T)e.x);
    const bool on = (base >> q) & 1u;
    br = on ? nr : br;
    bi = on ? ni : bi;
  }
  T ar[NA], ai[NA], hr[NB], hi[NB];
  ar[0] = T(1);
  ai[0] = T(0);
  hr[0] = br;
  hi[0] = bi;
#pragma unroll
  for (int k = 0; k < LOGV; ++k) {
    const float2 e = eq(__builtin_ctz(off(1 << k)));
    const T er = e.x, ei = e.y;
    if (k < LA) {
#pragma unroll
      for (int i = 0; i < (1 << k); ++i) {
        ar[i | (1 << k)] = fma(ar[i], er, -ai[i] * ei);
        ai[i | (1 << k)] = fma(ar[i], ei, ai[i] * er);
      }
    } else {
      const int kb = k - LA;
#pragma unroll
      for (int i = 0; i < (1 << kb); ++i) {
        hr[i | (1 << kb)] = fma(hr[i], er, -hi[i] * ei);
        hi[i | (1 << kb)] = fma(hr[i], ei, hi[i] * er);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < V; ++i) {
    const int ia = i & (NA - 1), ib = i >> LA;
    const T pr = fma(ar[ia], hr[ib], -ai[ia] * hi[ib]);
    const T pi = CONJ ? -fma(ar[ia], hi[ib], ai[ia] * hr[ib]) : fma(ar[ia], hi[ib], ai[ia] * hr[ib]);
    const T xr = x[i], xi = y[i];
    x[i] = fma(xr, pr, -xi * pi);
    y[i] = fma(xr, pi, xi * pr);
  }
}

// Phase sources for apply_gphase: scalar loads of the setting's coefficients (any block
// size), or a per-lane copy (lane q holds e_q; full wavefronts only) read out with
// readlane, which keeps the loop over the index bits free of memory waits.
struct PhaseLoad {
  cfptr um;
  __device__ float2 operator()(int q) const { return float2{uniform_f32(um[8 * q + 2]), uniform_f32(um[8 * q + 3])}; }
};
struct PhaseLanes {
  float2 v;
  __device__ float2 operator()(int q) const {
    return float2{__int_as_float(__builtin_amdgcn_readlane(__float_as_int(v.x), q)),
                  __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v.y), q))};
  }
};

// Orders the LDS accesses of a wavefront around an exchange between its lanes.
// A wavefront's LDS operations execute in issue order; the fences keep the
// compiler from reordering accesses across this point and emit no instruction.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Index-bit mask of the Y qubits of a decoded setting: bit 2b of t marks code 1 at
// index bit b, then the even bits are gathered into bits [0, 32) by halving steps.
// Codes above the n qubits are zero (X), so n needs no special handling.
__device__ __forceinline__ uint32_t ymask_of(uint64_t pc, int /*n*/) {
  uint64_t t = pc & ~(pc >> 1) & 0x5555555555555555ull;
  t = (t | (t >> 1)) & 0x3333333333333333ull;
  t = (t | (t >> 2)) & 0x0F0F0F0F0F0F0F0Full;
  t = (t | (t >> 4)) & 0x00FF00FF00FF00FFull;
  t = (t | (t >> 8)) & 0x0000FFFF0000FFFFull;
  t = (t | (t >> 16)) & 0x00000000FFFFFFFFull;
  return __builtin_amdgcn_readfirstlane((uint32_t)t);
}

// Y phase of one register layout.  Register i of a thread holds index base | off(i)
// with off linear in the bits of i, so the exponent is k = mt + popcount(i & m5):
// mt = popcount(base & ym) varies per lane, m5 marks the register bits whose index
// bit belongs to a Y qubit.  Three lane masks describe k mod 4:
//   sw = [k odd],  a = [k mod 4 in {2,3}],  b = [(k + 1) mod 4 in {2,3}].
// The forward phase (-i)^k exchanges the components where k is odd and negates x'
// where a, y' where b; the conjugate (+i)^k negates x' where b and y' where a.
// Visiting the registers in Gray-code order changes popcount(i & m5) by at most one
// per step; the masks then follow with a few scalar instructions:
//   k -> k + 1 :  sw' = ~sw,  a' = b,  b' = ~a
//   k -> k - 1 :  sw' = ~sw,  a' = ~b, b' = a
struct PhaseMasks {
  uint64_t sw, a, b;
};

__device__ __forceinline__ PhaseMasks phase_masks(uint32_t mt) {
  PhaseMasks m;
  m.sw = __builtin_amdgcn_ballot_w64((mt & 1u) != 0u);
  m.a = __builtin_amdgcn_ballot_w64((mt & 2u) != 0u);
  m.b = __builtin_amdgcn_ballot_w64(((mt + 1u) & 2u) != 0u);
  return m;
}

// Phase of one register with the current masks (four v_cndmask, the negation as a
// source modifier).
template <bool CONJ>
__device__ __forceinline__ void phase_apply(float& x, float& y, const PhaseMasks& m) {
  float xs, ys, xo, yo;
  const uint64_t nx = CONJ ? m.b : m.a;
  const uint64_t ny = CONJ ? m.a : m.b;
  asm("v_cndmask_b32_e64 %[xs], %[x], %[y], %[sw]\n\t"
      "v_cndmask_b32_e64 %[ys], %[y], %[x], %[sw]\n\t"
      "v_cndmask_b32_e64 %[xo], %[xs], -%[xs], %[nx]\n\t"
      "v_cndmask_b32_e64 %[yo], %[ys], -%[ys], %[ny]"
      : [xs] "=&v"(xs), [ys] "=&v"(ys), [xo] "=v"(xo), [yo] "=v"(yo)
      : [x] "v"(x), [y] "v"(y), [sw] "s"(m.sw), [nx] "s"(nx), [ny] "s"(ny));
  x = xo;
  y = yo;
}

// One Gray-code step over register bit K (UP: the bit is being set) followed by the
// phase of the register reached.  Scalar update and vector selects sit in one block
// so that the masks of all registers are never live at once.
template <int K, bool UP, bool CONJ>
__device__ __forceinline__ void phase_step(float& x, float& y, PhaseMasks& m, uint64_t m5) {
  uint64_t sw1, a1, b1, t;
  float xs, ys, xo, yo;
#define QST_PHASE_VALU(NX, NY)                                   \
  "v_cndmask_b32_e64 %[xs], %[x], %[y], %[sw1]\n\t"            \
  "v_cndmask_b32_e64 %[ys], %[y], %[x], %[sw1]\n\t"            \
  "v_cndmask_b32_e64 %[xo], %[xs], -%[xs], %[" NX "]\n\t"      \
  "v_cndmask_b32_e64 %[yo], %[ys], -%[ys], %[" NY "]"
#define QST_PHASE_OPS                                                                          \
  : [sw1] "=&s"(sw1), [a1] "=&s"(a1), [b1] "=&s"(b1), [t] "=&s"(t), [xs] "=&v"(xs), [ys] "=&v"(ys), \
    [xo] "=v"(xo), [yo] "=v"(yo)                                                               \
  : [x] "v"(x), [y] "v"(y), [sw] "s"(m.sw), [a] "s"(m.a), [b] "s"(m.b), [m5] "s"(m5), [k] "i"(K)  \
  : "scc"
#define QST_PHASE_UP                      \
  "s_not_b64 %[t], %[a]\n\t"             \
  "s_bitcmp1_b64 %[m5], %[k]\n\t"        \
  "s_cselect_b64 %[a1], %[b], %[a]\n\t"  \
  "s_cselect_b64 %[b1], %[t], %[b]\n\t"  \
  "s_cselect_b64 %[t], -1, 0\n\t"        \
  "s_xor_b64 %[sw1], %[sw], %[t]\n\t"
#define QST_PHASE_DOWN                    \
  "s_not_b64 %[t], %[b]\n\t"             \
  "s_bitcmp1_b64 %[m5], %[k]\n\t"        \
  "s_cselect_b64 %[a1], %[t], %[a]\n\t"  \
  "s_cselect_b64 %[b1], %[a], %[b]\n\t"  \
  "s_cselect_b64 %[t], -1, 0\n\t"        \
  "s_xor_b64 %[sw1], %[sw], %[t]\n\t"
  if constexpr (UP && !CONJ) asm(QST_PHASE_UP QST_PHASE_VALU("a1", "b1") QST_PHASE_OPS);
  if constexpr (UP && CONJ) asm(QST_PHASE_UP QST_PHASE_VALU("b1", "a1") QST_PHASE_OPS);
  if constexpr (!UP && !CONJ) asm(QST_PHASE_DOWN QST_PHASE_VALU("a1", "b1") QST_PHASE_OPS);
  if constexpr (!UP && CONJ) asm(QST_PHASE_DOWN QST_PHASE_VALU("b1", "a1") QST_PHASE_OPS);
#undef QST_PHASE_VALU
#undef QST_PHASE_OPS
#undef QST_PHASE_UP
#undef QST_PHASE_DOWN
  x = xo;
  y = yo;
  m.sw = sw1;
  m.a = a1;
  m.b = b1;
}

constexpr int gray(int j) { return j ^ (j >> 1); }
constexpr int ctz_c(int j) { return (j & 1) ? 0 : 1 + ctz_c(j >> 1); }

template <int J, int LOGV, bool CONJ>
__device__ __forceinline__ void phase_walk(float (&x)[1 << LOGV], float (&y)[1 << LOGV], PhaseMasks& m,
                                           uint64_t m5) {
  if constexpr (J < (1 << LOGV)) {
    constexpr int K = ctz_c(J);
    constexpr int I = gray(J);
    phase_step<K, ((I >> K) & 1) != 0, CONJ>(x[I], y[I], m, m5);
    phase_walk<J + 1, LOGV, CONJ>(x, y, m, m5);
  }
}

// FP64 form: exponent per element, k = mt + mi (mi uniform per register).
template <bool CONJ>
__device__ __forceinline__ void rot_k(double& x, double& y, uint32_t kk) {
  const bool sw = (kk & 1u) != 0u;
  const double xs = sw ? y : x;
  const double ys = sw ? x : y;
  const bool n_a = (kk & 2u) != 0u;
  const bool n_b = ((kk + 1u) & 2u) != 0u;
  x = (CONJ ? n_b : n_a) ? -xs : xs;
  y = (CONJ ? n_a : n_b) ? -ys : ys;
}

// Code word of the layout `lo` for the bits [from, to) of the block, where
// block bit q is index bit gbit0 + (q - qbase) of the state (q >= qbase).
// Bits outside [from, to) are skipped.
template <int LOGV>
__device__ __forceinline__ uint32_t layout_codes(uint64_t pc, int lo, int from, int to, int qbase, int gbit0) {
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < LOGV; ++k) {
    const int q = lo + k;
    uint32_t ck = CODE_SKIP;
    if (q >= from && q < to) ck = (uint32_t)((pc >> (2 * (gbit0 + q - qbase))) & 3ull);
    c |= ck << (2 * k);
  }
  return __builtin_amdgcn_readfirstlane(c);
}

// Number of non-Z qubits of a decoded setting (codes were clamped to <= 2).
__device__ __forceinline__ int nonz_count(uint64_t pc, int n) {
  const uint64_t odd = 0x5555555555555555ull;
  const uint64_t zbits = (pc >> 1) & odd;  // 1 where the code is 2 (Z)
  return n - __popcll(zbits);
}

// A setting's code word through the constant address space: with a uniform index the load is a
// scalar load, counted apart from the vector loads in flight (waiting for it then does not wait
// for a prefetch issued before it).
__device__ __forceinline__ uint64_t load_code(const uint64_t* pc, int b) {
  using cu64ptr = const __attribute__((address_space(4))) uint64_t*;
  const int bu = __builtin_amdgcn_readfirstlane(b);
  return ((cu64ptr)(pc))[bu];
}

__device__ __forceinline__ uint64_t uniform_u64(uint64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// ---------------------------------------------------------------- buffer access
// Global traffic of the staged kernels goes through raw buffer instructions:
// one resource (uniform base, byte size as bound) per array, one VGPR byte
// offset per thread shared by all of a thread's elements, and the per-element
// part as a uniform SGPR offset.  Out-of-range offsets read zero and drop
// writes, so a wrong index cannot reach memory outside the array.
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int RSRC_WORD3 = 0x00020000;  // gfx9-family raw buffer descriptor word 3

__device__ __forceinline__ rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, RSRC_WORD3);
}

using u32x2 = __attribute__((ext_vector_type(2))) unsigned int;
using u32x4 = __attribute__((ext_vector_type(4))) unsigned int;

__device__ __forceinline__ void bload(float2& v, rsrc_t rs, uint32_t voff, uint32_t soff) {
  v = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ void bload(double2& v, rsrc_t rs, uint32_t voff, uint32_t soff) {
  v = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ void bstore(const float2& v, rsrc_t rs, uint32_t voff, uint32_t soff) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), rs, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ void bstore(const double2& v, rsrc_t rs, uint32_t voff, uint32_t soff) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), rs, (int)voff, (int)soff, 0);
}

// Component forms: real and imaginary part in separate registers, the vector
// assembled and split here (no aggregate temporaries in private memory).
__device__ __forceinline__ void bload2(float& x, float& y, rsrc_t rs, uint32_t voff, uint32_t soff) {
  const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)voff, (int)soff, 0);
  x = __uint_as_float(v.x);
  y = __uint_as_float(v.y);
}
__device__ __forceinline__ void bload2(double& x, double& y, rsrc_t rs, uint32_t voff, uint32_t soff) {
  const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)voff, (int)soff, 0);
  x = __hiloint2double((int)v.y, (int)v.x);
  y = __hiloint2double((int)v.w, (int)v.z);
}
__device__ __forceinline__ void bstore2(float x, float y, rsrc_t rs, uint32_t voff, uint32_t soff) {
  u32x2 v;
  v.x = __float_as_uint(x);
  v.y = __float_as_uint(y);
  __builtin_amdgcn_raw_buffer_store_b64(v, rs, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ void bstore2(double x, double y, rsrc_t rs, uint32_t voff, uint32_t soff) {
  const unsigned long long bx = (unsigned long long)__double_as_longlong(x);
  const unsigned long long by = (unsigned long long)__double_as_longlong(y);
  u32x4 v;
  v.x = (uint32_t)bx;
  v.y = (uint32_t)(bx >> 32);
  v.z = (uint32_t)by;
  v.w = (uint32_t)(by >> 32);
  __builtin_amdgcn_raw_buffer_store_b128(v, rs, (int)voff, (int)soff, 0);
}

// BF16 storage of intermediate amplitudes: one complex number per 32-bit word,
// real part in the low half, each rounded to nearest even (finite values).
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t bf16_pack(float x, float y) {
  const f32x2_t v = {x, y};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_t));
}
__device__ __forceinline__ void bload2h(float& x, float& y, rsrc_t rs, uint32_t voff, uint32_t soff) {
  const uint32_t w = __builtin_amdgcn_raw_buffer_load_b32(rs, (int)voff, (int)soff, 0);
  x = __uint_as_float(w << 16);
  y = __uint_as_float(w & 0xffff0000u);
}
__device__ __forceinline__ void bstore2h(float x, float y, rsrc_t rs, uint32_t voff, uint32_t soff) {
  __builtin_amdgcn_raw_buffer_store_b32(bf16_pack(x, y), rs, (int)voff, (int)soff, 0);
}
// Load or store a complex number kept in BF16 (H16) or in the working precision.
template <bool H16, typename T>
__device__ __forceinline__ void ld_cs(T& x, T& y, rsrc_t rs, uint32_t voff, uint32_t soff) {
  if constexpr (H16)
    bload2h(x, y, rs, voff, soff);
  else
    bload2(x, y, rs, voff, soff);
}
template <bool H16, typename T>
__device__ __forceinline__ void st_cs(T x, T y, rsrc_t rs, uint32_t voff, uint32_t soff) {
  if constexpr (H16)
    bstore2h(x, y, rs, voff, soff);
  else
    bstore2(x, y, rs, voff, soff);
}

// Layout chain of a block of 2^NB amplitudes with 2^LOGV registers per thread:
// lo(0) = NB - LOGV, then LOGV bits lower per step down to 0.
template <int NB, int LOGV>
struct Chain {
  static constexpr int nb() { return NB; }
  static constexpr int lo(int k) {
    int l = NB - LOGV;
    for (int j = 0; j < k; ++j) l = l - LOGV > 0 ? l - LOGV : 0;
    return l;
  }
  static constexpr int count() {
    int k = 1;
    while (lo(k - 1) > 0) ++k;
    return k;
  }
  // first block bit handled by layout k (bits [lo(k), top(k)) are new there)
  static constexpr int top(int k) { return k == 0 ? NB : lo(k - 1); }
};

}  // namespace qst
