// Kernel templates of the staged butterfly path (gfx950).
//
// Forward map and adjoint of the atomic Born map over Pauli settings
// (eqs. atomic-born-map, qst-loss, likelihood-ratio-vector, weight-gradient,
// atom-wirtinger-gradient).  For setting b the rotation V_b = (x)_j V_{s_bj}
// factors over index bits; it is applied in the phase-split form of
// qst_device.hpp: one per-element Y phase plus one 4-operation butterfly per
// qubit, with the exact scale 2^(-k_b) (k_b = non-Z count) put on |phi|^2.
//
// A state of D = 2^n amplitudes is split into low bits [0, n_lo) and high bits
// [n_lo, n).  Per batch of S settings:
//   stage A  (tile, high bits)   X[s][r] = M_high P psi_r   (P: all Y phases; psi tile kept for S settings)
//   stage B  (chunk, low bits)   phi = M_low X;  p = 2^-k sum_r alpha_r |phi_r|^2;
//                                loss, g = dL/dp;  weight-gradient partials;
//                                W[s][r] = M_low (alpha_r 2^-k g * phi_r)
//   stage C  (tile, high bits)   grad_r += sum_s P^dagger M_high W[s][r]
// Stage B holds all R atoms of a chunk on chip, so p, g and the adjoint are
// fused; stages A and C amortise the psi read and the gradient
// read-modify-write over the S settings of a batch.  When n = n_lo the state
// is one chunk and stage B applies the phases itself.  All reductions are
// written to per-work-group slots and summed in a fixed order (deterministic).
#pragma once
#include "qst_device.hpp"
#include "qst_internal.hpp"

namespace qst {

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

// The same transpose when all threads of an atom sit in one wavefront: one plane
// takes the real and then the imaginary part.  LDS operations of a wavefront
// complete in issue order, so only the compiler has to be kept from moving
// them across the exchange points (wavefront-scope fences, no instructions).
template <int LOGV, int LO_FROM, int LO_TO, typename T>
__device__ __forceinline__ void lds_transpose_wave(T (&x)[1 << LOGV], T (&y)[1 << LOGV], T* pl, int tau) {
  T* w = pl + pad_base<LOGV, LO_FROM>(tau);
  const T* r = pl + pad_base<LOGV, LO_TO>(tau);
#pragma unroll
  for (int i = 0; i < (1 << LOGV); ++i) w[pad_off<LO_FROM>(i)] = x[i];
  wave_sync();
#pragma unroll
  for (int i = 0; i < (1 << LOGV); ++i) x[i] = r[pad_off<LO_TO>(i)];
  wave_sync();
#pragma unroll
  for (int i = 0; i < (1 << LOGV); ++i) w[pad_off<LO_FROM>(i)] = y[i];
  wave_sync();
#pragma unroll
  for (int i = 0; i < (1 << LOGV); ++i) y[i] = r[pad_off<LO_TO>(i)];
  wave_sync();
}

// Index bits that select the wavefront of a thread in layout `lo` of a vector of 2^NB
// amplitudes held by 2^(NB-LOGV) threads: thread bits 6 and up, which stand for index bit t
// below lo and t + LOGV from lo on.
template <int NB, int LOGV>
constexpr uint32_t wave_index_bits(int lo) {
  uint32_t m = 0;
  for (int t = 6; t < NB - LOGV; ++t) m |= 1u << (t < lo ? t : t + LOGV);
  return m;
}

// 2^14 amplitudes, 32 per thread (layouts 9, 4, 0): wavefronts hold index bits 6..8 in the
// first layout and 11..13 in the other two, so only the step 9 -> 4 crosses wavefronts.
static_assert(wave_index_bits<14, 5>(9) == 0x1C0u && wave_index_bits<14, 5>(4) == 0x3800u &&
              wave_index_bits<14, 5>(0) == 0x3800u);
// 16 per thread (layouts 10, 6, 2, 0): bits 6..9, then 10..13 from layout 6 on.
static_assert(wave_index_bits<14, 4>(10) == 0x3C0u && wave_index_bits<14, 4>(6) == 0x3C00u &&
              wave_index_bits<14, 4>(2) == 0x3C00u && wave_index_bits<14, 4>(0) == 0x3C00u);
// One wavefront per vector (2^11 amplitudes, 32 per thread): no wavefront bits.
static_assert(wave_index_bits<11, 5>(6) == 0u && wave_index_bits<11, 5>(0) == 0u);

// A work-group transpose between two layouts in which every wavefront holds the same index
// bits: each wavefront reads back only what it wrote, so the exchange needs no barrier.
// TAIL (the last transpose of a chain) ends with one all the same, so that whatever follows
// the chain finds the planes free, as after a work-group transpose.
template <int LOGV, int LO_FROM, int LO_TO, bool TAIL, typename T>
__device__ __forceinline__ void lds_transpose_own(T (&x)[1 << LOGV], T (&y)[1 << LOGV], T* re, T* im, int tau) {
  T* rw = re + pad_base<LOGV, LO_FROM>(tau);
  T* iw = im + pad_base<LOGV, LO_FROM>(tau);
#pragma unroll
  for (int i = 0; i < (1 << LOGV); ++i) {
    rw[pad_off<LO_FROM>(i)] = x[i];
    iw[pad_off<LO_FROM>(i)] = y[i];
  }
  wave_sync();
  const T* rr = re + pad_base<LOGV, LO_TO>(tau);
  const T* ir = im + pad_base<LOGV, LO_TO>(tau);
#pragma unroll
  for (int i = 0; i < (1 << LOGV); ++i) {
    x[i] = rr[pad_off<LO_TO>(i)];
    y[i] = ir[pad_off<LO_TO>(i)];
  }
  if constexpr (TAIL)
    __syncthreads();
  else
    wave_sync();
}

// Transpose of a layout chain: wavefront-local (one plane per atom, re = that plane),
// work-group wide between layouts that keep each wavefront's index bits (no barrier inside),
// or work-group wide (separate re and im planes, barriers after the writes and the reads).
// A work-group transpose that follows one of the second kind within a chain writes exactly
// the positions its wavefront has just read, so it needs no barrier before its writes.
template <bool WL, int NB, int LOGV, int LO_FROM, int LO_TO, bool TAIL, typename T>
__device__ __forceinline__ void lo_transpose(T (&x)[1 << LOGV], T (&y)[1 << LOGV], T* re, T* im, int tau) {
  if constexpr (WL)
    lds_transpose_wave<LOGV, LO_FROM, LO_TO>(x, y, re, tau);
  else if constexpr (wave_index_bits<NB, LOGV>(LO_FROM) == wave_index_bits<NB, LOGV>(LO_TO))
    lds_transpose_own<LOGV, LO_FROM, LO_TO, TAIL>(x, y, re, im, tau);
  else
    lds_transpose<LOGV, LO_FROM, LO_TO>(x, y, re, im, tau);
}

// Register bits of layout K of a chain that are new there (bits [lo(K), top(K))).
template <typename CH, int K>
constexpr uint32_t chain_mask() {
  uint32_t m = 0;
  for (int k = 0; k < 5; ++k)
    if (CH::lo(K) + k < CH::top(K)) m |= 1u << k;
  return m;
}

// Butterflies of every layout of the chain, first to last.  GEN: the general 2x2
// matrices of the setting (um, by index bit) instead of the Pauli butterflies.  SYNC_END
// = false leaves out the barrier that ends a chain whose last transpose keeps each
// wavefront's index bits: allowed when every wavefront's next access to the planes is the
// first transpose of an adjoint chain (which writes only the positions it has just read).
template <int K, typename CH, bool WL, bool GEN, int LOGV, bool SYNC_END = true, typename T>
__device__ __forceinline__ void fwd_chain(T (&x)[1 << LOGV], T (&y)[1 << LOGV], T* re, T* im, int tau, uint64_t pc,
                                          cfptr um) {
  if constexpr (K < CH::count()) {
    if constexpr (K > 0)
      lo_transpose<WL, CH::nb(), LOGV, CH::lo(K - 1), CH::lo(K), SYNC_END && K + 1 == CH::count()>(x, y, re, im, tau);
    if constexpr (GEN)
      xform_gen<LOGV, false, chain_mask<CH, K>()>(x, y, um, CH::lo(K));
    else
      xform_xz<LOGV, chain_mask<CH, K>()>(x, y, layout_codes<LOGV>(pc, CH::lo(K), CH::lo(K), CH::top(K), 0, 0));
    fwd_chain<K + 1, CH, WL, GEN, LOGV, SYNC_END>(x, y, re, im, tau, pc, um);
  }
}

// The adjoint butterflies from the last layout back to layout 0 (the Pauli ones are
// their own adjoints; the general ones take the conjugate transpose).
template <int K, typename CH, bool WL, bool GEN, int LOGV, typename T>
__device__ __forceinline__ void adj_chain(T (&x)[1 << LOGV], T (&y)[1 << LOGV], T* re, T* im, int tau, uint64_t pc,
                                          cfptr um) {
  if constexpr (GEN)
    xform_gen<LOGV, true, chain_mask<CH, K>()>(x, y, um, CH::lo(K));
  else
    xform_xz<LOGV, chain_mask<CH, K>()>(x, y, layout_codes<LOGV>(pc, CH::lo(K), CH::lo(K), CH::top(K), 0, 0));
  if constexpr (K > 0) {
    lo_transpose<WL, CH::nb(), LOGV, CH::lo(K), CH::lo(K - 1), K == 1>(x, y, re, im, tau);
    adj_chain<K - 1, CH, WL, GEN, LOGV>(x, y, re, im, tau, pc, um);
  }
}

// Apply the Y phase (or its conjugate) to the registers of one layout: register i
// of this thread holds index base_index | off(i), off(i) uniform and linear in the
// bits of i, so the exponent is popcount(base & ym) (per lane) + popcount(i & m5)
// with m5 the register bits that land on Y qubits.
template <bool CONJ, int LOGV, typename T, typename OffFn>
__device__ __forceinline__ void apply_phase(T (&x)[1 << LOGV], T (&y)[1 << LOGV], uint32_t base_index, uint32_t ym,
                                            OffFn off) {
  const uint32_t mt = (uint32_t)__popc(base_index & ym);
  if constexpr (std::is_same<T, float>::value) {
    uint32_t m5 = 0;
#pragma unroll
    for (int k = 0; k < LOGV; ++k) m5 |= (off(1 << k) & ym) != 0u ? (1u << k) : 0u;
    PhaseMasks m = phase_masks(mt);
    phase_apply<CONJ>(x[0], y[0], m);
    phase_walk<1, LOGV, CONJ>(x, y, m, (uint64_t)__builtin_amdgcn_readfirstlane(m5));
  } else {
#pragma unroll
    for (int i = 0; i < (1 << LOGV); ++i) {
      const uint32_t mi = __builtin_amdgcn_readfirstlane((uint32_t)__popc(off(i) & ym));
      rot_k<CONJ>(x[i], y[i], mt + mi);
    }
  }
}

// ------------------------------------------------------------------ stage B
// Persistent low stage: work-group w takes chunks w, w + G, w + 2G, ... of the
// batch (chunk = one setting x 2^n_lo consecutive outcomes, all atoms) and
// prefetches the next chunk's amplitudes and data row while it works on the
// current one.  Its loss and weight-gradient partials go to one slot per
// (batch, work-group), so the final sums do not depend on timing.
// PHASE: the state is one chunk (n = n_lo): the input is the atoms and this stage
// applies the Y phases.  H16: the setting-batch intermediates X (input, when the state
// has high bits) and W (output) are stored in BF16; arithmetic stays in T.  GEN:
// general local settings (a rotation per qubit, the input-side phase where the state
// enters and leaves the rotations, scale 1).
// Register bits per thread of the low stage (lo_logv_of): the forward pass over staged
// chunks of 2^12 and more outcomes takes 2^4 values per thread and up to 1024 threads per
// work-group, twice the wavefronts to overlap its loads and barriers.  The adjoint keeps
// 2^5 values: with 1024 threads its registers would spill.
template <int N_LO, bool PHASE, bool ADJ>
constexpr int lo_logv() {
  return lo_logv_of(N_LO, !PHASE, ADJ);
}
template <int N_LO, bool PHASE, bool ADJ>
constexpr int lo_max_threads() {
  return lo_logv<N_LO, PHASE, ADJ>() == 4 ? 1024 : 512;
}

template <typename T, int N_LO, bool ADJ, bool PHASE, bool H16, bool GEN = false>
__global__ __launch_bounds__((lo_max_threads<N_LO, PHASE, ADJ>())) void k_stage_lo(const LoBatch m) {
  using C2 = cx<T>;
  constexpr int LOGV = lo_logv<N_LO, PHASE, ADJ>();
  constexpr int V = 1 << LOGV;
  constexpr int U = 1 << N_LO;
  constexpr int UPAD = U + (U >> 5);
  constexpr int LOG_TA = N_LO - LOGV;
  constexpr int TA = 1 << LOG_TA;
  constexpr int NPF = 2;  // data-row values prefetched per thread
  using CH = Chain<N_LO, LOGV>;
  constexpr int NL = CH::count();
  constexpr int LO0 = CH::lo(0);
  constexpr bool H16_IN = H16 && !PHASE;                      // X in BF16 (atoms are read as given)
  constexpr uint32_t CBI = H16_IN ? 4u : (uint32_t)sizeof(C2);  // bytes per input complex
  constexpr uint32_t CBO = H16 ? 4u : (uint32_t)sizeof(C2);     // bytes per output complex
  constexpr bool WL = LOG_TA <= 6;  // the threads of one atom form (part of) one wavefront
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  const int atom = tid >> LOG_TA;
  const int tau = tid & (TA - 1);
  const int G = gridDim.x;
  const int RM = m.rmax;

  // LDS (sized for the largest rank of the launch), wavefront-local transposes (WL):
  // one plane of UPAD entries per atom, then the table alpha_r |phi_r|^2 [R][UPAD]
  // and the sensitivity row g [UPAD].  Otherwise: a real and an imaginary plane per
  // atom, with the table and g aliasing the first R+1 rows (barriers separate their
  // uses from the transposes).
  T* planes = reinterpret_cast<T*>(smem);
  T* re = WL ? planes + (size_t)atom * UPAD : planes + (size_t)atom * 2 * UPAD;
  T* im = WL ? re : re + UPAD;
  T* qb = WL ? planes + (size_t)RM * UPAD : planes;
  T* gb = qb + (size_t)RM * UPAD;
  const size_t plane_rows = WL ? 2 * (size_t)RM + 1 : 2 * (size_t)RM;
  double* red = reinterpret_cast<double*>(smem + (((plane_rows * UPAD * sizeof(T)) + 15) & ~(size_t)15));

  const uint32_t pos0 = (uint32_t)lay_pos<LOGV>(tau, 0, LO0);
  // Instance of a chunk of the launch (the chunks of instance k are [begin[k], begin[k+1])).
  auto inst_of = [&](int c) {
    int k = 0;
    while (k + 1 < m.count && c >= m.begin[k + 1]) ++k;
    return k;
  };
  // Buffer extent of one chunk (all atoms of the instance) in plain order.
  auto extent = [&](const LoArgs& a, uint32_t cb) { return (uint32_t)(((long long)(a.R - 1) * a.D + U) * cb); };

  double loss_acc = 0.0, h_acc = 0.0;
  T al_cur = T(0);         // this thread's atom weight in the current instance
  int cur = -1;            // instance whose partials are being accumulated
  uint32_t touched = 0u;   // instances this work-group wrote partials for

  // Partials of instance k for this work-group: loss in row 0, h_r in rows 1..R.
  auto flush = [&](int k) {
    const LoArgs& a = m.a[k];
    touched |= 1u << k;
    const long long slot = a.slot_base + blockIdx.x;
    if (a.part != nullptr) {
      if (ADJ) {
        red[tid] = h_acc;
        __syncthreads();
        for (int st = TA >> 1; st > 0; st >>= 1) {
          if (tau < st) red[tid] += red[tid + st];
          __syncthreads();
        }
        if (tau == 0 && atom < a.R) a.part[(long long)(1 + atom) * a.nslots + slot] = red[tid];
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
        __syncthreads();
      }
    }
    loss_acc = 0.0;
    h_acc = 0.0;
  };

  // Two register buffers take turns: chunk c + G is fetched into one while chunk c is
  // transformed in the other.  A buffer holds each amplitude's real and imaginary parts in
  // adjacent registers, so every 64-bit load lands where the body reads it (with separate
  // real and imaginary arrays the compiler moves the halves apart right after the load and
  // has to wait for it there, which serialises the fetch with the work).  Every fetch is
  // issued, also past the last chunk (then through an empty buffer range, which reads
  // zeros): a fetch under a condition makes the compiler's waits cover it at once.
  T bp[2 * V], bpf[NPF], bq[2 * V], bqf[NPF];
  auto issue = [&](int c_in, T (&bb)[2 * V], T (&bf)[NPF]) __attribute__((always_inline)) {
    const bool valid = c_in < m.total;
    const int c = valid ? c_in : (m.total > 0 ? m.total - 1 : 0);
    const int k = inst_of(c);
    const LoArgs& a = m.a[k];
    const int cl = c - m.begin[k];
    const int s = cl >> a.n_hi;
    const int h = cl & ((1 << a.n_hi) - 1);
    // X position of chunk element l: index bits [xb, N_LO) above the high bits (xb = N_LO:
    // plain order, and always when the input is the atoms)
    const int xb = N_LO - a.x_up;
    auto xpos = [&](uint32_t l) { return ((l >> xb) << (a.n_hi + xb)) | (l & ((1u << xb) - 1u)); };
    const unsigned char* sbase = reinterpret_cast<const unsigned char*>(a.src) +
                                 ((long long)s * a.src_set_stride + ((long long)h << xb)) * CBI;
    // threads of atoms beyond this instance's rank lie outside the extent: they read zeros
    const uint32_t ext = a.x_up ? (uint32_t)(((long long)a.R * a.D - ((long long)h << xb)) * CBI) : extent(a, CBI);
    const rsrc_t rs = make_rsrc(sbase, valid ? ext : 0u);
    const uint32_t vo0 = (uint32_t)(((long long)atom * a.D + xpos(pos0)) * CBI);
#pragma unroll
    for (int i = 0; i < V; ++i) ld_cs<H16_IN>(bb[2 * i], bb[2 * i + 1], rs, vo0, xpos((uint32_t)(i << LO0)) * CBI);
    if (valid && (a.grad_p != nullptr || (a.loss_kind != 2 && a.fidx == nullptr))) {
      const long long row = (long long)(a.b0 + s) * a.D + ((long long)h << N_LO);
#pragma unroll
      for (int j = 0; j < NPF; ++j) {
        const int u = tid + j * nthr;
        bf[j] = 0;
        if (u < U) bf[j] = a.grad_p ? reinterpret_cast<const T*>(a.grad_p)[row + u] : (T)a.freqs[row + u];
      }
    }
  };

  // The body is inlined once per register buffer; every multiply-add in it is an
  // explicit fma and implicit contraction is off, so both copies round alike and a
  // chunk's results do not depend on which buffer (or which work-group) takes it.
  auto body = [&](int c, const T (&bb)[2 * V], const T (&bf)[NPF]) __attribute__((always_inline)) {
#pragma clang fp contract(off)
    T x[V], y[V];
#pragma unroll
    for (int i = 0; i < V; ++i) {
      x[i] = bb[2 * i];
      y[i] = bb[2 * i + 1];
    }
    const int k = inst_of(c);
    if (k != cur) {
      if (cur >= 0) flush(cur);
      cur = k;
      // loaded when the instance changes, not per chunk: a vector load here would have to
      // wait for the next chunk's prefetch, which is issued before it
      al_cur = atom < m.a[k].R ? (T)m.a[k].alpha[atom] : T(0);
    }
    const LoArgs& a = m.a[k];
    const int cl = c - m.begin[k];
    const int s = cl >> a.n_hi;
    const int h = cl & ((1 << a.n_hi) - 1);
    const int b = a.b0 + s;
    const long long D = a.D;
    const T al = al_cur;
    const uint64_t pc = load_code(a.pc, b);
    const T s2 = GEN ? T(1) : (T)ldexp(1.0, -nonz_count(pc, a.n));
    const cfptr um = GEN ? to_const(a.um + (size_t)b * a.n * 8) : nullptr;
    const double Bd = (double)a.B;
    const float inv_b = (float)(1.0 / Bd);
    const float eps_f = (float)a.eps;
    const bool row_data = a.grad_p != nullptr || a.loss_kind != 2;
    T fv[NPF];
#pragma unroll
    for (int j = 0; j < NPF; ++j) fv[j] = bf[j];

    uint32_t ym = 0;
    if constexpr (PHASE && !GEN) {
      ym = ymask_of(pc, a.n);
      apply_phase<false, LOGV>(x, y, pos0, ym, [](int i) { return (uint32_t)(i << LO0); });
    }
    if constexpr (PHASE && GEN)
      apply_gphase<false, LOGV>(x, y, pos0, a.n, [](int i) { return (uint32_t)(i << LO0); }, PhaseLoad{um});
    fwd_chain<0, CH, WL, GEN, LOGV>(x, y, re, im, tau, pc, um);
    // Final layout is lo = 0: alpha_r |phi_r|^2 into LDS, reduced over atoms per outcome.
    T* qrow = qb + (size_t)atom * UPAD + pad_base<LOGV, 0>(tau);
#pragma unroll
    for (int i = 0; i < V; ++i) qrow[pad_off<0>(i)] = al * fma(x[i], x[i], y[i] * y[i]);
    __syncthreads();
    const long long row = (long long)b * D + ((long long)h << N_LO);
    const T* gp = reinterpret_cast<const T*>(a.grad_p);
    const T* pbp = reinterpret_cast<const T*>(a.pbase);
    // Sparse frequencies: this chunk's observed outcomes are scattered into the g row
    // (zero elsewhere); each outcome's thread reads its value before writing g there.
    // Every thread has passed the barrier above, so no read of the previous chunk's g
    // is pending.  Outcomes outside the chunk are dropped.
    const bool sparse = a.fidx != nullptr && gp == nullptr && a.loss_kind != 2;
    if (sparse) {
      for (int u = tid; u < U; u += nthr) gb[pad32(u)] = T(0);
      __syncthreads();
      const long long ci = (long long)b * (1ll << a.n_hi) + h;
      const long long e0 = a.fchunk[ci];
      long long e1 = a.fchunk[ci + 1];
      if (e1 < e0) e1 = e0;
      for (long long e = e0 + tid; e < e1; e += nthr) {
        const long long uu = (long long)a.fidx[e] - ((long long)h << N_LO);
        if (uu >= 0 && uu < U) gb[pad32((int)uu)] = (T)a.freqs[e];
      }
      __syncthreads();
    }
    // One outcome u of the chunk: p (atom sum, scale, base), loss term, sensitivity.
    // d is the data value of the outcome (dL/dp in the generic mode, else the frequency).
    auto outcome = [&](int u, T d, T pb) __attribute__((always_inline)) {
      T p = 0;
      for (int r = 0; r < a.R; ++r) p += qb[(size_t)r * UPAD + pad32(u)];
      p *= s2;
      if (pbp) p += pb;
      if (a.probs) reinterpret_cast<T*>(a.probs)[row + u] = p;
      T g = 0;
      if (gp) {
        g = d;
      } else if constexpr (std::is_same<T, float>::value) {
        // FP32 path: p carries single-precision rounding already, so each term is
        // formed in FP32 (hardware log2 and reciprocal, about 1 ulp) and summed in FP64.
        if (a.loss_kind == 0) {
          if (d > 0.0f) {
            const float fb = d * inv_b;
            const float piv = fmaf(p, inv_b, eps_f);
            loss_acc -= (double)(fb * (__builtin_amdgcn_logf(piv) * 0.693147180559945309f));
            g = -(fb * inv_b) * __builtin_amdgcn_rcpf(piv);
          }
        } else if (a.loss_kind == 1) {
          const float rr = (p - d) * inv_b;
          loss_acc += (double)(0.5f * rr * rr);
          g = rr * inv_b;
        }
      } else if (a.loss_kind == 0) {
        const double f = (double)d;
        if (f > 0.0) {
          const double piv = (double)p / Bd + a.eps;
          loss_acc -= (f / Bd) * log(piv);
          g = (T)(-(f / Bd) / piv / Bd);
        }
      } else if (a.loss_kind == 1) {
        const double rr = ((double)p - (double)d) / Bd;
        loss_acc += 0.5 * rr * rr;
        g = (T)(rr / Bd);
      }
      if (a.gneg) reinterpret_cast<T*>(a.gneg)[row + u] = -g;
      if (ADJ) gb[pad32(u)] = g * s2;
    };
    // This thread's outcomes are u = tid + j * nthr.  The first NPF data values were
    // prefetched with the chunk; the rest (and the base values) are loaded in groups of
    // NG whose loads are all in flight before the first of them is used.
    constexpr int NG = 4;
    // Dense data without base probabilities: the first NPF outcomes take their data from the
    // chunk's prefetch, so nothing here waits for memory (a wait on a load issued after the
    // next chunk's prefetch would wait for that prefetch too).
    int j_first = 0;
    if (!sparse && pbp == nullptr) {
#pragma unroll
      for (int jj = 0; jj < NPF; ++jj) {
        const int u = tid + jj * nthr;
        if (u < U) outcome(u, row_data ? fv[jj] : T(0), T(0));
      }
      j_first = NPF;
    }
    for (int j0 = j_first; tid + j0 * nthr < U; j0 += NG) {
      T dg[NG], bg[NG];
#pragma unroll
      for (int jj = 0; jj < NG; ++jj) {
        const int u = tid + (j0 + jj) * nthr;
        dg[jj] = 0;
        bg[jj] = 0;
        if (u < U) {
          if (sparse) {
            dg[jj] = gb[pad32(u)];
          } else if (row_data) {
            if (jj < NPF && j0 == 0)  // only when the prefetched outcomes were not taken above
              dg[jj] = fv[jj < NPF ? jj : 0];
            else
              dg[jj] = gp ? gp[row + u] : (T)a.freqs[row + u];
          }
          if (pbp) bg[jj] = pbp[row + u];
        }
      }
#pragma unroll
      for (int jj = 0; jj < NG; ++jj) {
        const int u = tid + (j0 + jj) * nthr;
        if (u < U) outcome(u, dg[jj], bg[jj]);
      }
    }
    __syncthreads();
    if (ADJ) {
      T hl = 0;
#pragma unroll
      for (int i = 0; i < V; ++i) {
        const T gv = gb[pad_base<LOGV, 0>(tau) + pad_off<0>(i)];
        hl = fma(gv, fma(x[i], x[i], y[i] * y[i]), hl);
        const T sc = al * gv;
        x[i] *= sc;
        y[i] *= sc;
      }
      h_acc += (double)hl;
      if constexpr (!WL) __syncthreads();  // every thread has read g before the planes are reused
      adj_chain<NL - 1, CH, WL, GEN, LOGV>(x, y, re, im, tau, pc, um);
      if constexpr (PHASE && !GEN) apply_phase<true, LOGV>(x, y, pos0, ym, [](int i) { return (uint32_t)(i << LO0); });
      if constexpr (PHASE && GEN)
        apply_gphase<true, LOGV>(x, y, pos0, a.n, [](int i) { return (uint32_t)(i << LO0); }, PhaseLoad{um});
      // W position of chunk element l: index bits [wb, N_LO) go above the high bits
      const int wb = N_LO - a.w_up;
      auto wpos = [&](uint32_t l) { return ((l >> wb) << (a.n_hi + wb)) | (l & ((1u << wb) - 1u)); };
      unsigned char* dbase = reinterpret_cast<unsigned char*>(a.dst) + ((long long)s * a.R * D + ((long long)h << wb)) * CBO;
      // atoms beyond the instance's rank fall outside the range: their stores are dropped
      const rsrc_t rd =
          make_rsrc(dbase, a.w_up ? (uint32_t)(((long long)a.R * D - ((long long)h << wb)) * CBO) : extent(a, CBO));
      const uint32_t vo0 = (uint32_t)(((long long)atom * D + wpos(pos0)) * CBO);
#pragma unroll
      for (int i = 0; i < V; ++i) st_cs<H16>(x[i], y[i], rd, vo0, wpos((uint32_t)(i << LO0)) * CBO);
      if constexpr (!WL) __syncthreads();
    }
  };
  issue(blockIdx.x, bp, bpf);
  for (int c = blockIdx.x; c < m.total; c += 2 * G) {
    issue(c + G, bq, bqf);
    body(c, bp, bpf);
    if (c + G >= m.total) break;
    issue(c + 2 * G, bp, bpf);
    body(c + G, bq, bqf);
  }
  if (cur >= 0) flush(cur);
  // Instances this work-group had no chunk of: zero partials, so every slot is defined.
  for (int k = 0; k < m.count; ++k) {
    if ((touched >> k) & 1u) continue;
    const LoArgs& a = m.a[k];
    if (a.part == nullptr) continue;
    const long long slot = a.slot_base + blockIdx.x;
    if (ADJ && tau == 0 && atom < a.R) a.part[(long long)(1 + atom) * a.nslots + slot] = 0.0;
    if (tid == 0 && a.grad_p == nullptr && a.loss_kind != 2) a.part[slot] = 0.0;
  }
}

template <typename T, int N_LO, bool PHASE, bool H16, bool GEN = false>
hipError_t launch_lo_n(const Geometry& g, const LoBatch& m, bool adjoint, hipStream_t st) {
  const int logv = adjoint ? lo_logv<N_LO, PHASE, true>() : lo_logv<N_LO, PHASE, false>();
  const int nthr = m.rmax << (N_LO - logv);
  const size_t lds = lo_lds_bytes_logv(g, logv);
  const unsigned grid = (unsigned)g.grid_lo;
  if (adjoint) {
    {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_stage_lo<T, N_LO, true, PHASE, H16, GEN>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    k_stage_lo<T, N_LO, true, PHASE, H16, GEN><<<grid, nthr, lds, st>>>(m);
  } else {
    {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_stage_lo<T, N_LO, false, PHASE, H16, GEN>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    k_stage_lo<T, N_LO, false, PHASE, H16, GEN><<<grid, nthr, lds, st>>>(m);
  }
  return hipGetLastError();
}

template <typename T, int N_LO, bool PHASE, bool H16, bool GEN = false>
int lo_occupancy_n(const Geometry& g) {
  constexpr int LOGV = lo_logv<N_LO, PHASE, true>();
  const int nthr = g.R << (N_LO - LOGV);
  const size_t lds = lo_lds_bytes_logv(g, LOGV);
  if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_stage_lo<T, N_LO, true, PHASE, H16, GEN>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return 1;
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_stage_lo<T, N_LO, true, PHASE, H16, GEN>, nthr, lds) !=
      hipSuccess)
    return 1;
  return blocks > 0 ? blocks : 1;
}

// ------------------------------------------------------------------ stages A and C
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

// H16: X (forward output) and W (adjoint input) are stored in BF16.  GEN: general
// local settings (the input-side phase of every bit, then the rotations of the high bits;
// the adjoint in reverse order).
template <int TB, int N_HI, bool ADJ, bool H16, bool GEN = false>
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
  extern __shared__ __align__(16) unsigned char smem[];
  T* re = reinterpret_cast<T*>(smem);
  T* im = re + NPAD;
  const int tid = threadIdx.x;
  const int n_lo = a.n_lo;
  const int ncb = 1 << (n_lo - C);
  // work-group = (tile, split); a split takes settings [s_lo, s_hi) of the batch
  const int sp = blockIdx.x % a.nsplit;
  const int tile = blockIdx.x / a.nsplit;
  const int r = tile / ncb;
  const int cb = tile - r * ncb;
  const int s_lo = (int)((long long)sp * a.S / a.nsplit);
  const int s_hi = (int)((long long)(sp + 1) * a.S / a.nsplit);
  const long long D = a.D;
  const uint32_t cbase = (uint32_t)cb << C;  // index of the tile origin within the atom
  const long long origin = (long long)r * D + cbase;
  const uint32_t vbytes = (uint32_t)((D - cbase) * CB);
  constexpr uint32_t CBH = H16 ? 4u : CB;  // bytes per complex of X and W
  const uint32_t t0 = tile_off(lay_pos<LOGV>(tid, 0, LO0), C, n_lo);
  const uint32_t tf = tile_off(lay_pos<LOGV>(tid, 0, LOF), C, n_lo);
  const uint32_t vo0 = t0 * CB;
  const uint32_t vof = tf * CB;
  auto off0 = [=](int i) { return tile_off((uint32_t)i << LO0, C, n_lo); };
  auto offf = [=](int i) { return tile_off((uint32_t)i << LOF, C, n_lo); };
  // X (forward output) and W (adjoint input) may be stored with index bits [wb, n_lo) above
  // the high bits (the low stage uses the same order), so a tile's rows lie 2^wb elements
  // apart (wb = n_lo: plain layout, wb >= C).
  const int wb = n_lo - a.w_up;
  const uint32_t cphys = ((cbase >> wb) << (a.n_hi + wb)) | (cbase & ((1u << wb) - 1u));
  const long long origin_w = (long long)r * D + cphys;
  const uint32_t vbytes_w = (uint32_t)((D - cphys) * CBH);
  const uint32_t t0w = tile_off(lay_pos<LOGV>(tid, 0, LO0), C, wb);
  const uint32_t tfw = tile_off(lay_pos<LOGV>(tid, 0, LOF), C, wb);
  auto off0w = [=](int i) { return tile_off((uint32_t)i << LO0, C, wb); };
  auto offfw = [=](int i) { return tile_off((uint32_t)i << LOF, C, wb); };

  // General settings: lane q of every wavefront holds the phase e_q of the setting
  // (fetched one setting ahead) for the per-element phase.
  const int lane = tid & 63;
  auto lane_e = [&](int s) -> float2 {
    float2 e{0.f, 0.f};
    if (lane < a.n) e = *reinterpret_cast<const float2*>(a.um + ((size_t)(a.b0 + s) * a.n + lane) * 8 + 2);
    return e;
  };

  if (!ADJ) {
    const rsrc_t rs = make_rsrc(reinterpret_cast<const C2*>(a.src) + origin, vbytes);
    T kx[V], ky[V];
#pragma unroll
    for (int i = 0; i < V; ++i) {
      bload2(kx[i], ky[i], rs, vo0, off0(i) * CB);
    }
    float2 ecur{0.f, 0.f};
    if constexpr (GEN) {
      if (s_lo < s_hi) ecur = lane_e(s_lo);
    }
    for (int s = s_lo; s < s_hi; ++s) {
      const uint64_t pc = load_code(a.pc, a.b0 + s);
      T x[V], y[V];
#pragma unroll
      for (int i = 0; i < V; ++i) {
        x[i] = kx[i];
        y[i] = ky[i];
      }
      if constexpr (GEN) {
        float2 enxt = ecur;
        if (s + 1 < s_hi) enxt = lane_e(s + 1);
        // register bit k of layout lo is index bit n_lo + lo + k - C
        const cfptr um = to_const(a.um + (size_t)(a.b0 + s) * a.n * 8);
        apply_gphase<false, LOGV>(x, y, cbase | t0, a.n, off0, PhaseLanes{ecur});
        ecur = enxt;
        xform_gen<LOGV, false, M0>(x, y, um, n_lo + LO0 - C);
        if constexpr (TWO) {
          lds_transpose<LOGV, LO0, LO1>(x, y, re, im, tid);
          xform_gen<LOGV, false, M1>(x, y, um, n_lo + LO1 - C);
        }
      } else {
        apply_phase<false, LOGV>(x, y, cbase | t0, ymask_of(pc, a.n), off0);
        xform_xz<LOGV, M0>(x, y, layout_codes<LOGV>(pc, LO0, LO0, TB, C, n_lo));
        if constexpr (TWO) {
          lds_transpose<LOGV, LO0, LO1>(x, y, re, im, tid);
          xform_xz<LOGV, M1>(x, y, layout_codes<LOGV>(pc, LO1, LO1, LO0, C, n_lo));
        }
      }
      const rsrc_t rx =
          make_rsrc(reinterpret_cast<unsigned char*>(a.dst) + ((long long)s * a.R * D + origin_w) * CBH, vbytes_w);
#pragma unroll
      for (int i = 0; i < V; ++i) st_cs<H16>(x[i], y[i], rx, tfw * CBH, offfw(i) * CBH);
    }
  } else {
    T ax[V], ay[V];
#pragma unroll
    for (int i = 0; i < V; ++i) ax[i] = ay[i] = T(0);
    // Two register buffers take turns: the next setting's W tile is fetched into one
    // while the other is transformed in place.  Every fetch is issued unconditionally (a
    // setting past the split reads zeros through an empty buffer range): the number of
    // loads in flight is then the same on every path into a use, so the compiler's wait
    // there covers only the buffer in use.  A fetch under a condition made the waits
    // assume the path without it and retire the prefetch too, every second setting.
    T px[V], py[V], qx[V], qy[V];
    float2 pe{0.f, 0.f}, qe{0.f, 0.f};
    auto issue = [&](int s, T (&bx)[V], T (&by)[V], float2& be) __attribute__((always_inline)) {
      const bool valid = s < s_hi;
      const int sv = valid ? s : s_lo;
      const rsrc_t rw = make_rsrc(
          reinterpret_cast<const unsigned char*>(a.src) + ((long long)sv * a.R * D + origin_w) * CBH, valid ? vbytes_w : 0u);
#pragma unroll
      for (int i = 0; i < V; ++i) {
        ld_cs<H16>(bx[i], by[i], rw, t0w * CBH, off0w(i) * CBH);
      }
      if constexpr (GEN) {
        if (valid) be = lane_e(s);
      }
    };
    auto body = [&](int s, T (&x)[V], T (&y)[V], const float2& e) __attribute__((always_inline)) {
      if constexpr (GEN) {
        const cfptr um = to_const(a.um + (size_t)(a.b0 + s) * a.n * 8);
        xform_gen<LOGV, true, M0>(x, y, um, n_lo + LO0 - C);
        if constexpr (TWO) {
          lds_transpose<LOGV, LO0, LO1>(x, y, re, im, tid);
          xform_gen<LOGV, true, M1>(x, y, um, n_lo + LO1 - C);
        }
        apply_gphase<true, LOGV>(x, y, cbase | tf, a.n, offf, PhaseLanes{e});
      } else {
        const uint64_t pc = load_code(a.pc, a.b0 + s);
        const uint32_t ym = ymask_of(pc, a.n);
        xform_xz<LOGV, M0>(x, y, layout_codes<LOGV>(pc, LO0, LO0, TB, C, n_lo));
        if constexpr (TWO) {
          lds_transpose<LOGV, LO0, LO1>(x, y, re, im, tid);
          xform_xz<LOGV, M1>(x, y, layout_codes<LOGV>(pc, LO1, LO1, LO0, C, n_lo));
        }
        apply_phase<true, LOGV>(x, y, cbase | tf, ym, offf);
      }
#pragma unroll
      for (int i = 0; i < V; ++i) {
        ax[i] += x[i];
        ay[i] += y[i];
      }
    };
    // General settings keep the conditional fetches: their per-lane phases make the
    // unconditional form run out of registers (160 spilled), which costs far more than
    // the early waits.
    constexpr bool UNCOND = !GEN;
    if (UNCOND || s_lo < s_hi) issue(s_lo, px, py, pe);
    for (int s = s_lo; s < s_hi; s += 2) {
      if (UNCOND || s + 1 < s_hi) issue(s + 1, qx, qy, qe);
      body(s, px, py, pe);
      if (s + 1 < s_hi) {
        if (UNCOND || s + 2 < s_hi) issue(s + 2, px, py, pe);
        body(s + 1, qx, qy, qe);
      }
    }
    // one split: accumulate into the gradient; several: this split's sum to its slice.  The
    // gradient tile's loads are all issued before the first is used (the condition is uniform,
    // so it is tested once rather than around every load).
    const bool whole = a.nsplit == 1;
    C2* out = whole ? reinterpret_cast<C2*>(a.dst) : reinterpret_cast<C2*>(a.part) + (long long)sp * a.R * D;
    const rsrc_t rg = make_rsrc(out + origin, vbytes);
    if (whole && !a.first) {
      T gx[V], gy[V];
#pragma unroll
      for (int i = 0; i < V; ++i) bload2(gx[i], gy[i], rg, vof, offf(i) * CB);
#pragma unroll
      for (int i = 0; i < V; ++i) {
        ax[i] += gx[i];
        ay[i] += gy[i];
      }
    }
#pragma unroll
    for (int i = 0; i < V; ++i) bstore2(ax[i], ay[i], rg, vof, offf(i) * CB);
  }
}

template <int TB, int N_HI, bool H16, bool GEN = false>
hipError_t launch_hi_n(const Geometry& g, const HiArgs& a, bool adjoint, hipStream_t st) {
  const int nthr = 1 << (TB - 5);
  const size_t lds = hi_lds_bytes(g);
  const unsigned grid = (unsigned)((g.R << (g.n_lo - g.c)) * a.nsplit);
  if (adjoint) {
    {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_stage_hi<TB, N_HI, true, H16, GEN>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    k_stage_hi<TB, N_HI, true, H16, GEN><<<grid, nthr, lds, st>>>(a);
  } else {
    {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_stage_hi<TB, N_HI, false, H16, GEN>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    k_stage_hi<TB, N_HI, false, H16, GEN><<<grid, nthr, lds, st>>>(a);
  }
  return hipGetLastError();
}

}  // namespace qst
