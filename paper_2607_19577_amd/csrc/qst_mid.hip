// The middle pass of the three-pass schedule and its instantiations: tiles of 2^14 amplitudes
// with 1..10 rows, FP32 or BF16 intermediates, Pauli or general settings.  It shares the tile
// machinery (layouts, LDS transposes, tile offsets) of stages A and C in qst_stages.hpp.
#include "qst_stages.hpp"

namespace qst {

// ------------------------------------------------------------------ middle pass
// Three-pass schedule: when the bits above the low stage do not fit one tile, index bits
// [row_lo, row_lo + N_ROWS) get a pass of their own between stage A and the low stage (on X)
// and between the low stage and stage C (on W).  A tile is 2^N_ROWS rows (those bits) by 2^C
// contiguous columns (index bits 0 .. C-1); its other index bits, [C, row_lo) and
// [row_lo + N_ROWS, n), and the atom name it.  Per setting of the work-group's share the tile
// is rotated in registers (one LDS transpose when the rows reach below the first layout) and
// written back in place; the next setting's tile is fetched meanwhile, unconditionally (past
// the share it reads zeros through an empty range), as in stage C.  The rotations of different
// bits commute, so this pass may run between the other two in either direction; it applies no
// phases (stage A and stage C apply them for every bit).  ADJ matters for general settings only
// (the Pauli butterflies are their own adjoints).
template <int TB, int N_ROWS, bool ADJ, bool H16, bool GEN = false>
__global__ __launch_bounds__(512) void k_stage_mid(const MidArgs a) {
  using T = float;
  constexpr int LOGV = 5;
  constexpr int V = 1 << LOGV;
  constexpr int C = TB - N_ROWS;
  constexpr int LO0 = TB - LOGV;
  constexpr bool TWO = C < LO0;
  constexpr int LO1 = TB - 2 * LOGV > 0 ? TB - 2 * LOGV : 0;
  constexpr int LOF = TWO ? LO1 : LO0;
  constexpr uint32_t M0 = rows_mask(LO0, C, TB);
  constexpr uint32_t M1 = rows_mask(LO1, C, LO0);
  constexpr int NPAD = (1 << TB) + (1 << (TB - 5));
  constexpr uint32_t CBH = H16 ? 4u : 8u;  // bytes per complex of X and W
  extern __shared__ __align__(16) unsigned char smem[];
  T* re = reinterpret_cast<T*>(smem);
  T* im = re + NPAD;
  const int tid = threadIdx.x;
  const int row_lo = a.row_lo;
  const int nlow = row_lo - C;              // tile-naming bits between the columns and the rows
  const int sp = blockIdx.x % a.nsplit;
  const long long tile = blockIdx.x / a.nsplit;
  const int nname = a.n - N_ROWS - C;       // tile-naming index bits in all
  const int r = (int)(tile >> nname);
  const long long rest = tile & ((1ll << nname) - 1);
  const long long cbl = rest & ((1ll << nlow) - 1);
  const long long cbh = rest >> nlow;
  const long long origin = (cbh << (row_lo + N_ROWS)) | (cbl << C);  // tile origin within the atom
  const int s_lo = (int)((long long)sp * a.S / a.nsplit);
  const int s_hi = (int)((long long)(sp + 1) * a.S / a.nsplit);
  const long long D = a.D;
  const uint32_t vbytes = (uint32_t)((D - origin) * CBH);
  const uint32_t t0 = tile_off(lay_pos<LOGV>(tid, 0, LO0), C, row_lo);
  const uint32_t tf = tile_off(lay_pos<LOGV>(tid, 0, LOF), C, row_lo);
  auto off0 = [=](int i) { return tile_off((uint32_t)i << LO0, C, row_lo); };
  auto offf = [=](int i) { return tile_off((uint32_t)i << LOF, C, row_lo); };
  auto tile_base = [&](int s) {
    return reinterpret_cast<unsigned char*>(a.buf) + ((long long)s * a.R * D + (long long)r * D + origin) * CBH;
  };
  T px[V], py[V], qx[V], qy[V];
  auto issue = [&](int s, T (&bx)[V], T (&by)[V]) __attribute__((always_inline)) {
    const bool valid = s < s_hi;
    const rsrc_t rs = make_rsrc(tile_base(valid ? s : s_lo), valid ? vbytes : 0u);
#pragma unroll
    for (int i = 0; i < V; ++i) ld_cs<H16>(bx[i], by[i], rs, t0 * CBH, off0(i) * CBH);
  };
  auto body = [&](int s, T (&x)[V], T (&y)[V]) __attribute__((always_inline)) {
    if constexpr (GEN) {
      const cfptr um = to_const(a.um + (size_t)(a.b0 + s) * a.n * 8);
      xform_gen<LOGV, ADJ, M0>(x, y, um, row_lo + LO0 - C);
      if constexpr (TWO) {
        lds_transpose<LOGV, LO0, LO1>(x, y, re, im, tid);
        xform_gen<LOGV, ADJ, M1>(x, y, um, row_lo + LO1 - C);
      }
    } else {
      const uint64_t pc = load_code(a.pc, a.b0 + s);
      xform_xz<LOGV, M0>(x, y, layout_codes<LOGV>(pc, LO0, LO0, TB, C, row_lo));
      if constexpr (TWO) {
        lds_transpose<LOGV, LO0, LO1>(x, y, re, im, tid);
        xform_xz<LOGV, M1>(x, y, layout_codes<LOGV>(pc, LO1, LO1, LO0, C, row_lo));
      }
    }
    const rsrc_t rw = make_rsrc(tile_base(s), vbytes);
#pragma unroll
    for (int i = 0; i < V; ++i) st_cs<H16>(x[i], y[i], rw, tf * CBH, offf(i) * CBH);
  };
  issue(s_lo, px, py);
  for (int s = s_lo; s < s_hi; s += 2) {
    issue(s + 1, qx, qy);
    body(s, px, py);
    if (s + 1 < s_hi) {
      issue(s + 2, px, py);
      body(s + 1, qx, qy);
    }
  }
}

template <int TB, int N_ROWS, bool H16, bool GEN = false>
hipError_t launch_mid_n(const Geometry& g, const MidArgs& a, bool adjoint, hipStream_t st) {
  const size_t lds = hi_lds_bytes(g);
  const long long tiles = (long long)g.R << (g.n - N_ROWS - (TB - N_ROWS));
  const unsigned grid = (unsigned)(tiles * a.nsplit);
  if (adjoint) {
    {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_stage_mid<TB, N_ROWS, true, H16, GEN>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    k_stage_mid<TB, N_ROWS, true, H16, GEN><<<grid, 512, lds, st>>>(a);
  } else {
    {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_stage_mid<TB, N_ROWS, false, H16, GEN>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    k_stage_mid<TB, N_ROWS, false, H16, GEN><<<grid, 512, lds, st>>>(a);
  }
  return hipGetLastError();
}


hipError_t launch_stage_mid(const Geometry& g, const MidArgs& a, bool adjoint, hipStream_t st) {
  if (g.elem != 4 || a.t != 14 || a.rows != g.n_mid || a.c != a.t - a.rows || a.c > a.row_lo || a.nsplit < 1 ||
      a.nsplit > a.S || a.row_lo + a.rows > g.n)
    return hipErrorInvalidValue;
  if (g.gen && (g.h16 || a.um == nullptr)) return hipErrorInvalidValue;
#define QST_MID(NRv)                                                                  \
  if (a.rows == NRv) {                                                                \
    if (g.gen) return launch_mid_n<14, NRv, false, true>(g, a, adjoint, st);          \
    return g.h16 ? launch_mid_n<14, NRv, true>(g, a, adjoint, st)                     \
                 : launch_mid_n<14, NRv, false>(g, a, adjoint, st);                   \
  }
  QST_MID(1) QST_MID(2) QST_MID(3) QST_MID(4) QST_MID(5)
  QST_MID(6) QST_MID(7) QST_MID(8) QST_MID(9) QST_MID(10)
#undef QST_MID
  return hipErrorInvalidValue;
}

}  // namespace qst
