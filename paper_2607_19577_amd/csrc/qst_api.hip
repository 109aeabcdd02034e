// Host side of the C ABI declared in include/qst.h: validation, geometry and
// workspace planning, the per-batch launch sequence, and the host-orchestrated
// spectral refactorisation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "qst.h"
#include "qst_internal.hpp"

using qst::Geometry;

// Scratch of the no-allocation backward (qst_backward_static): a fixed device array, one
// copy per GPU, held until the process ends.  In host code this name is only a symbol
// for hipGetSymbolAddress; the device address of each GPU's copy is looked up once per
// device (scratch_address) and only that address is passed to kernels.
constexpr size_t kStaticScratchBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

struct qst_handle {
  int device = 0;
  int num_cu = 256;
  hipStream_t stream = nullptr;
  std::string last_error;
  void* ws = nullptr;  // workspace arena (grow-only)
  size_t ws_bytes = 0;
  std::vector<void*> retired;  // outgrown arenas, freed by qst_destroy (captured graphs may still use them)
  int* dflag = nullptr;  // device flag raised by kernels (OR of 1: bad code, 2: table entry not unitary)
  int* hflag = nullptr;  // pinned host copy
  hipEvent_t flag_ev = nullptr;
  bool flag_pending = false;
  // implementation choices per shape (n, R, B rounded up to a power of two, path) and routing
  // policies per call signature (qst_plan with autotune, qst_plan_choice)
  std::map<std::tuple<int, int, int, int>, qst_choice> choices;
  std::map<uint64_t, std::pair<int, int>> policies;  // signature -> (onchip mode, fused slices)
  std::pair<int, int> cur_policy{-1, -1};            // policy of the call being run
  std::string arch;
  std::map<std::tuple<int, int, int, int>, int> occupancy;  // (n_lo, n_hi > 0, R, elem) -> low-stage WGs per CU
  std::map<std::pair<int, int>, int> oc_occupancy;           // (n, adjoint) -> on-chip pass WGs per CU
  // stage timing
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_next = 0;
  struct Mark {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Mark> marks;
  int open_kind = -1;
  bool prof_outer = false;  // a whole G v product is bracketed: its stages are not
  int gv_occupancy = 0;     // work-groups per CU of the grouped G v low stage
  hipEvent_t open_ev = nullptr;
  // no-allocation mode (qst_backward_static): ws points at the device's static scratch
  void* static_scratch = nullptr;  // this device's copy of `scratch` (from qst_create)
  bool static_ws = false;
  // side streams (default priority) that the classes of a multi-instance call fork onto
  // from `stream` and join back from, through events (also under graph capture)
  static constexpr int kSide = 4;
  hipStream_t side[kSide] = {};
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev[kSide] = {};
  bool side_ok = false;
};

namespace {

constexpr int G1 = 256;  // first-level reduction width
// Largest rank: the low stage holds all R atoms of a chunk of at least 2^6 outcomes in one
// work-group of at most 512 threads (R 2^6 <= 2^14), and the reweight kernel takes R <= 1024.
constexpr int kMaxRank = 256;

enum { PK_DECODE = 0, PK_HI_FWD = 1, PK_LO = 2, PK_HI_ADJ = 3, PK_REDUCE = 4, PK_OTHER = 5, PK_GV = 6, PK_MID = 7 };
constexpr int kProfKinds = 8;

hipEvent_t prof_event(qst_handle* h) {
  if (h->ev_next == h->ev_pool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    h->ev_pool.push_back(e);
  }
  return h->ev_pool[h->ev_next++];
}

bool capturing(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess) return false;
  return cs != hipStreamCaptureStatusNone;
}

// Bracket the next launch(es) of one stage kind.
void prof_begin(qst_handle* h, int kind) {
  if (!h->prof || h->static_ws || h->prof_outer || capturing(h->stream)) return;
  hipEvent_t e = prof_event(h);
  if (!e || hipEventRecord(e, h->stream) != hipSuccess) return;
  h->open_kind = kind;
  h->open_ev = e;
}

void prof_end(qst_handle* h) {
  if (!h->prof || h->static_ws || h->prof_outer || h->open_kind < 0 || capturing(h->stream)) return;
  hipEvent_t e = prof_event(h);
  if (!e || hipEventRecord(e, h->stream) != hipSuccess) return;
  h->marks.push_back({h->open_kind, h->open_ev, e});
  h->open_kind = -1;
}

// Bracket one whole G v product of the refactor (the stages inside it are not bracketed).
void prof_outer_begin(qst_handle* h) {
  h->prof_outer = false;
  prof_begin(h, PK_GV);
  h->prof_outer = true;
}
void prof_outer_end(qst_handle* h) {
  h->prof_outer = false;
  prof_end(h);
}

qst_status set_err(qst_handle* h, qst_status s, const std::string& msg) {
  if (h) h->last_error = msg;
  return s;
}

#define QST_HIP(expr)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return set_err(h, QST_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));   \
  } while (0)


qst_status ensure_ws(qst_handle* h, size_t bytes) {
  if (bytes <= h->ws_bytes) return QST_OK;
  if (h->static_ws)
    return set_err(h, QST_ERR_SHAPE, "the call needs " + std::to_string(bytes) +
                                         " bytes of scratch; qst_backward_static holds " +
                                         std::to_string(kStaticScratchBytes) + " bytes");
  if (capturing(h->stream))
    return set_err(h, QST_ERR_CAPTURE, "workspace must grow while the stream is capturing; call qst_plan first");
  if (h->ws) {
    h->retired.push_back(h->ws);
    h->ws = nullptr;
    h->ws_bytes = 0;
  }
  size_t want = bytes + (bytes >> 3);
  if (hipMalloc(&h->ws, want) != hipSuccess) {
    h->ws = nullptr;
    return set_err(h, QST_ERR_OOM, "workspace allocation of " + std::to_string(want) + " bytes failed");
  }
  h->ws_bytes = want;
  return QST_OK;
}

int elem_of(qst_path p) { return p == QST_PATH_BUTTERFLY_F64 ? 8 : 4; }

bool path_valid(int p) { return p >= QST_PATH_AUTO && p <= QST_PATH_BUTTERFLY_BF16; }

// Paths that keep every (setting, atom) vector in HBM and make one pass per qubit
// (plain) or per group of four qubits (MFMA tiles).
bool pass_path(qst_path p) {
  return p == QST_PATH_PLAIN_F32 || p == QST_PATH_TILE_F16 || p == QST_PATH_TILE_BF16;
}

qst_path resolve(qst_path p) { return p == QST_PATH_AUTO ? QST_PATH_BUTTERFLY_F32 : p; }

// Tile bits of stage A (which = 0) and stage C (which = 1): QST_TILE_BITS_FWD and
// QST_TILE_BITS_ADJ (environment, read once) override the defaults for tuning.
int env_tile_bits(int which) {
  static const int v[2] = {[] {
                             const char* e = std::getenv("QST_TILE_BITS_FWD");
                             return e ? std::atoi(e) : 0;
                           }(),
                           [] {
                             const char* e = std::getenv("QST_TILE_BITS_ADJ");
                             return e ? std::atoi(e) : 0;
                           }()};
  return v[which];
}

int pow2_at_least(int x) {
  int p = 1;
  while (p < x && p < (1 << 30)) p <<= 1;
  return p;
}

std::tuple<int, int, int, int> shape_key(int n, int R, int B, qst_path path) {
  return std::make_tuple(n, R, pow2_at_least(B), (int)path);
}

// The handle's choice for a shape, or null.
const qst_choice* find_choice(const qst_handle* h, int n, int R, int B, qst_path path) {
  auto it = h->choices.find(shape_key(n, R, B, path));
  return it == h->choices.end() ? nullptr : &it->second;
}

// Geometry of the staged path for (n, R, B).
qst_status make_geometry(qst_handle* h, int n, int R, int B, qst_path path, Geometry& g) {
  const int elem = elem_of(path);
  g = Geometry{};
  g.h16 = path == QST_PATH_BUTTERFLY_BF16;
  g.n = n;
  g.R = R;
  g.B = B;
  g.D = 1ll << n;
  g.elem = elem;
  const long long cap = elem == 4 ? 16384 : 8192;  // amplitudes one low-stage work-group holds
  constexpr size_t kLdsMax = 160 * 1024;
  int n_lo = n;
  for (; n_lo > 0; --n_lo) {
    if (((long long)R << n_lo) > cap) continue;
    g.n_lo = n_lo;
    g.n_hi = n - n_lo;
    g.logv_lo = qst::lo_logv_of(n_lo, n_lo < n, true);
    if (qst::lo_lds_bytes(g) <= kLdsMax) break;  // the larger of the forward and the adjoint pass
  }
  if (n_lo < 1) return set_err(h, QST_ERR_SHAPE, "rank too large for the on-chip low stage");
  g.n_lo = n_lo;
  g.n_hi = n - n_lo;
  g.logv_lo = qst::lo_logv_of(n_lo, n_lo < n, true);
  if (g.n_hi > 10 && elem == 4) {
    // Three passes: the top bits for stages A and C, a middle pass for the rest; the split is
    // as even as the tile shapes allow (longer contiguous rows for both tile passes).
    const int lo_min = std::max(1, 14 - g.n_lo);  // a middle tile needs its 14 - rows columns below it
    g.n_mid = std::min(10, std::max(lo_min, g.n_hi / 2));
    const int top = g.n_hi - g.n_mid;
    if (top < 1 || top > 10)
      return set_err(h, QST_ERR_SHAPE,
                     "n=" + std::to_string(n) + ", R=" + std::to_string(R) + ": the bits above the low stage need more than three passes");
    g.c_mid = 14 - g.n_mid;
    g.t = g.t_adj = 14;
    g.c = g.c_adj = 14 - top;
    return QST_OK;
  }
  if (g.n_hi > 0) {
    if (elem != 4)
      return set_err(h, QST_ERR_UNSUPPORTED,
                     "the FP64 path holds the whole state on chip: needs R * 2^n <= 8192");
    auto tile_ok = [&](int t) {
      const int c = t - g.n_hi;
      const bool shape = (t == 14 && g.n_hi <= 10) || (t == 13 && g.n_hi <= 3) || (t == 12 && g.n_hi <= 2) ||
                         (t == 11 && g.n_hi == 1);
      return shape && c >= 0 && c <= g.n_lo;
    };
    g.t = std::min(n, env_tile_bits(0) > 0 ? env_tile_bits(0) : 14);
    g.t_adj = std::min(n, env_tile_bits(1) > 0 ? env_tile_bits(1) : 14);
    if (const qst_choice* c = find_choice(h, n, R, B, path)) {
      if (c->tile_bits_fwd > 0 && tile_ok(c->tile_bits_fwd)) g.t = c->tile_bits_fwd;
      if (c->tile_bits_adj > 0 && tile_ok(c->tile_bits_adj)) g.t_adj = c->tile_bits_adj;
    }
    if (!tile_ok(g.t) || !tile_ok(g.t_adj))
      return set_err(h, QST_ERR_UNSUPPORTED,
                     "n=" + std::to_string(n) + ", R=" + std::to_string(R) + " is outside the tile-stage shapes");
    g.c = g.t - g.n_hi;
    g.c_adj = g.t_adj - g.n_hi;
  }
  return QST_OK;
}

// The geometry as stages A and C see it: with a middle pass, their rows are the top
// n_hi - n_mid bits, starting at bit n_lo + n_mid (the bits below them name the tile).
Geometry top_view(const Geometry& g) {
  Geometry t = g;
  t.n_lo = g.n_lo + g.n_mid;
  t.n_hi = g.n_hi - g.n_mid;
  return t;
}

// Work-groups per tile of the high-bit stages: enough (tile, split) pairs for two per
// CU, each split with at least 8 settings of the batch.  (g: the stage's own view.)
int split_of(const qst_handle* h, const Geometry& g, int c, int S) {
  if (g.n_hi == 0) return 1;
  const long long tiles = (long long)g.R << (g.n_lo - c);
  const long long want = (2ll * h->num_cu + tiles - 1) / tiles;
  return (int)std::max(1ll, std::min(want, (long long)std::max(1, S / 8)));
}

// Persistent low-stage grid for batches of S settings.
void set_grid(qst_handle* h, Geometry& g, int S) {
  g.S = S;
  g.split_adj = split_of(h, top_view(g), g.c_adj, S);
  const long long chunks = (long long)S << g.n_hi;
  int per_cu = 1;
  if (h->device >= 0) {
    const auto key = std::make_tuple(g.n_lo, (g.n_hi > 0 ? 1 : 0) | (g.h16 ? 2 : 0) | (g.gen ? 4 : 0) | (g.lo2 ? 8 : 0),
                                     g.R, g.elem);
    auto it = h->occupancy.find(key);
    if (it == h->occupancy.end())
      it = h->occupancy.emplace(key, g.lo2 ? qst::lo2_occupancy(g) : qst::lo_blocks_per_cu(g)).first;
    per_cu = it->second;
  }
  const long long resident = (long long)h->num_cu * per_cu;
  g.grid_lo = (int)std::max(1ll, std::min(chunks, resident));
}

// Settings per batch.  QST_SETTINGS_PER_BATCH (environment, read once) overrides
// the default for tuning experiments.
int env_batch() {
  static const int v = [] {
    const char* e = std::getenv("QST_SETTINGS_PER_BATCH");
    return e ? std::max(0, std::atoi(e)) : 0;
  }();
  return v;
}

// Layout of the low stage's output W for the adjoint tile stage (two passes): its tiles read
// rows of 2^c_adj elements, 2^n_lo apart in plain order.  The low stage can store index bits
// [wb, n_lo) of each chunk above the high bits instead (LoArgs::w_up = n_lo - wb), so those
// rows lie 2^wb apart and neighbouring tiles share DRAM pages.  Measured at n=20, R=16,
// B=2000 (rows of 16 elements), ms per step (low stage, adjoint tile stage): wb = 10 (plain)
// 220.4 (113.1, 56.5); wb = 6 215.0 (114.1, 50.2); wb = 5 214.5 (114.3, 49.5); wb = 4 217.4
// (118.0, 48.7).  With BF16 intermediates: 162.4, 158.1, 156.3, 156.9.  Default: wb = 5 when
// the tile rows hold at most 32 elements, else plain.  The shape's choice (w_row_bits) or
// QST_W_ROW_BITS (environment, read once) override it.
int w_up_of(const qst_handle* h, const Geometry& g, qst_path path) {
  static const int env = [] {
    const char* e = std::getenv("QST_W_ROW_BITS");
    return e ? std::atoi(e) : 0;
  }();
  const int dflt = g.c_adj <= 5 ? std::min(5, g.n_lo) : g.n_lo;
  int wb = env > 0 ? env : dflt;
  if (const qst_choice* c = find_choice(h, g.n, g.R, g.B, path))
    if (c->w_row_bits > 0) wb = c->w_row_bits;
  if (wb < g.c_adj || wb > g.n_lo) wb = dflt;
  return g.n_lo - wb;
}

// Order of X between the forward tile stage and the low stage, as for W (LoArgs::x_up).
// Measured at n=20, R=16, B=2000 (rows of 16 elements), ms per step (forward tile stage, low
// stage): xb = 10 (plain) 215.1 (49.9, 115.2); xb = 6 213.9 (50.0, 114.0); xb = 5 229.0
// (52.3, 126.3); xb = 4 225.7 (51.0, 124.5).  With BF16 intermediates: 155.0, 151.6, 170.1,
// 191.8.  Default: xb = 6 when the tile rows hold at most 32 elements, else plain; the
// shape's choice (x_row_bits) or QST_X_ROW_BITS (environment, read once) override it.
int x_up_of(const qst_handle* h, const Geometry& g, qst_path path) {
  static const int env = [] {
    const char* e = std::getenv("QST_X_ROW_BITS");
    return e ? std::atoi(e) : 0;
  }();
  // (the two-sweep low stage reads each atom's part of a chunk whole: plain order, 268.6
  // against 272.4 ms per step at n=22, R=16, B=500 with rows 2^6 apart)
  const int dflt = (g.c <= 5 && !g.lo2) ? std::min(6, g.n_lo) : g.n_lo;
  int xb = env > 0 ? env : dflt;
  if (const qst_choice* c = find_choice(h, g.n, g.R, g.B, path))
    if (c->x_row_bits > 0) xb = c->x_row_bits;
  if (xb < g.c || xb > g.n_lo) xb = dflt;
  return g.n_lo - xb;
}

int default_S(const Geometry& g) {
  if (env_batch() > 0) return std::min(env_batch(), g.B);
  const long long per = (long long)g.R * g.D * 2 * g.elem;
  long long s = (16ll << 30) / std::max(per, 1ll);
  if (s < 1) s = 1;
  if (s > g.B) s = g.B;
  // X and W hold S settings each (16 GiB each at most, S = 128 at n=20, R=16).  Larger
  // batches amortise the psi read and the gradient update and need fewer launches
  // (measured at n=20, R=16, B=2000: S = 4 -> 337, 16 -> 253, 64 -> 220, 96 -> 218.7,
  // 128 -> 218.1 ms per step).
  return (int)s;
}

struct WsLayout {
  size_t pc, um, cptr, X, W, part, lvl1, sums, tan, gneg, split, total;
};

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

long long nslots_of(const Geometry& g, qst_path path) {
  if (pass_path(path)) return (long long)g.B * ((g.D + 255) / 256);
  const long long batches = (g.B + g.S - 1) / g.S;
  return batches * g.grid_lo;
}

WsLayout layout_ws(const Geometry& g, int S, qst_path path, bool with_gneg, size_t base = 0) {
  WsLayout L{};
  size_t o = base;
  const size_t vec = (size_t)S * g.R * g.D * 2 * (g.h16 ? 2 : g.elem);
  L.pc = o;
  o = al256(o + (size_t)g.B * 8);
  L.um = o;
  if (g.gen) o = al256(o + (size_t)g.B * g.n * 8 * sizeof(float));
  L.cptr = o;
  if (g.sparse) o = al256(o + ((size_t)g.B * (pass_path(path) ? 1 : (1ull << g.n_hi)) + 1) * 8);
  L.X = o;
  if (g.n_hi > 0 || pass_path(path)) o = al256(o + vec);
  L.W = o;
  if (!pass_path(path)) o = al256(o + vec);
  L.part = o;
  o = al256(o + (size_t)(g.R + 1) * nslots_of(g, path) * 8);
  L.lvl1 = o;
  o = al256(o + (size_t)(g.R + 1) * G1 * 8);
  L.sums = o;
  o = al256(o + (size_t)(g.R + 1) * 8);
  L.tan = o;
  o = al256(o + (size_t)g.R * G1 * 2 * 8 + (size_t)g.R * 2 * 8);
  L.gneg = o;
  if (with_gneg) o = al256(o + (size_t)g.B * g.D * g.elem);
  L.split = o;
  if (g.n_hi > 0 && g.split_adj > 1) o = al256(o + (size_t)g.split_adj * g.R * g.D * 2 * g.elem);
  L.total = o;
  return L;
}

qst_status check_flag(qst_handle* h) {
  if (!h->flag_pending || capturing(h->stream)) return QST_OK;
  if (hipEventQuery(h->flag_ev) != hipSuccess) return QST_OK;  // not reached yet: report later
  h->flag_pending = false;
  if (*h->hflag) {
    const int f = *h->hflag;
    *h->hflag = 0;
    if (qst::launch_fill(h->dflag, sizeof(int), h->stream) != hipSuccess)
      return set_err(h, QST_ERR_DEVICE, "clearing the device flag failed");
    std::string msg;
    if (f & 1) msg = "a setting held a code outside the Pauli codes and the unitary table";
    if (f & 2) msg += std::string(msg.empty() ? "" : "; ") + "a unitary table entry was not unitary to 1e-6";
    return set_err(h, QST_ERR_NUMERIC, msg + " (treated as the identity)");
  }
  return QST_OK;
}

void post_flag(qst_handle* h) {
  if (capturing(h->stream)) return;
  // a flag that cannot be fetched is not reported (the call's own status covers the failure)
  if (hipMemcpyAsync(h->hflag, h->dflag, sizeof(int), hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
      hipEventRecord(h->flag_ev, h->stream) != hipSuccess)
    return;
  h->flag_pending = true;
}

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

qst_status validate_instance(qst_handle* h, const qst_instance& in, qst_path path, bool need_freqs) {
  if (in.n_qubits < 1 || in.n_qubits > 30)
    return set_err(h, QST_ERR_SHAPE, "n_qubits must be in 1..30 (got " + std::to_string(in.n_qubits) + ")");
  if (in.rank < 1 || in.rank > kMaxRank)
    return set_err(h, QST_ERR_SHAPE, "rank must be in 1.." + std::to_string(kMaxRank));
  // one setting's R vectors are addressed through a 32-bit buffer range
  if (((long long)in.rank << in.n_qubits) * (path == QST_PATH_BUTTERFLY_F64 ? 16 : 8) > 0xFFFFFFFFll)
    return set_err(h, QST_ERR_SHAPE, "R * 2^n * (bytes per amplitude) must stay below 4 GiB");
  if (pass_path(path) && (in.n_qubits > 20 || in.rank > 16))
    return set_err(h, QST_ERR_UNSUPPORTED, "the plain and tile paths take n <= 20 and R <= 16");
  if (in.n_settings < 1) return set_err(h, QST_ERR_SHAPE, "n_settings must be >= 1");
  if (in.settings_per_batch < 0) return set_err(h, QST_ERR_SHAPE, "settings_per_batch must be >= 0");
  if (!in.atoms || !in.weights || !in.settings) return set_err(h, QST_ERR_INVALID_ARG, "null atoms/weights/settings");
  if (need_freqs && !in.freqs) return set_err(h, QST_ERR_INVALID_ARG, "freqs required for the requested loss");
  const size_t ea = path == QST_PATH_BUTTERFLY_F64 ? 16 : 8;
  if (!aligned(in.atoms, ea) || !aligned(in.weights, 8) || (in.freqs && !aligned(in.freqs, 4)) ||
      (in.probs_base && !aligned(in.probs_base, (size_t)elem_of(path))))
    return set_err(h, QST_ERR_ALIGN, "atoms/weights/freqs/probs_base not aligned to their element size");
  if (in.freqs_rowptr) {
    if (!in.freqs_index || !in.freqs) return set_err(h, QST_ERR_INVALID_ARG, "sparse frequencies need freqs and freqs_index");
    if (in.freqs_nnz < 0 || in.freqs_nnz > (long long)in.n_settings << in.n_qubits)
      return set_err(h, QST_ERR_SHAPE, "freqs_nnz must be in 0..B*D");
    if (!aligned(in.freqs_rowptr, 8) || !aligned(in.freqs_index, 4))
      return set_err(h, QST_ERR_ALIGN, "freqs_rowptr/freqs_index not aligned to their element size");
  }
  if (in.unitaries) {
    if (path != QST_PATH_BUTTERFLY_F32)
      return set_err(h, QST_ERR_UNSUPPORTED, "general local settings run on QST_PATH_BUTTERFLY_F32");
    if (in.n_unitaries < 1 || in.n_unitaries > 253) return set_err(h, QST_ERR_SHAPE, "n_unitaries must be in 1..253");
    if (!aligned(in.unitaries, 8)) return set_err(h, QST_ERR_ALIGN, "unitaries not 8-byte aligned");
  }
  return QST_OK;
}

// Enqueue the forward (adjoint=false) or fused forward+adjoint pipeline of one instance.
struct RunSpec {
  const qst_instance* in;
  qst_path path;
  qst_loss loss_kind;
  double eps;
  void* probs;
  double* loss;
  const void* grad_p;
  void* atom_grad;
  double* weight_grad;
  int project_tangent;
  void* gneg;  // optional: receives -dL/dp
  bool adjoint;
  int S_override;
};

// Per-instance options that change kernels or workspace: general settings, sparse data.
void mark(Geometry& g, const qst_instance& in) {
  g.gen = in.unitaries != nullptr;
  g.sparse = in.freqs_rowptr != nullptr;
  // More than ten bits above the low stage: with Pauli settings and dense data the low stage
  // takes n - 10 bits with its atoms looped (two sweeps over X), which keeps two tile passes
  // and moves 24 B per (setting, atom) amplitude less than a middle pass would.  QST_LO2=0
  // (environment, read once) keeps the middle pass.
  static const bool lo2_on = [] {
    const char* e = std::getenv("QST_LO2");
    return !(e && std::atoi(e) == 0);
  }();
  if (lo2_on && g.n_mid > 0 && !g.gen && !g.sparse && g.elem == 4 && g.n - 10 >= 10 && g.n - 10 <= 14) {
    g.lo2 = true;
    g.n_lo = g.n - 10;
    g.n_hi = 10;
    g.n_mid = g.c_mid = 0;
    g.t = g.t_adj = 14;
    g.c = g.c_adj = 4;
    g.logv_lo = g.n_lo <= 10 ? 4 : 5;
  }
}

// Settings per batch of one instance: the override, else the caller's choice, the
// autotuned value or the default, in that order.
int batch_size(const qst_handle* h, const Geometry& g, const qst_instance& in, qst_path path, int S_override) {
  if (S_override > 0) return std::min(S_override, g.B);
  if (in.settings_per_batch > 0) return std::min((int)in.settings_per_batch, g.B);
  if (const qst_choice* c = find_choice(h, g.n, g.R, g.B, path))
    if (c->settings_per_batch > 0) return std::min((int)c->settings_per_batch, g.B);
  return default_S(g);
}

// No-allocation mode: the largest batch size up to S whose workspace fits the static
// scratch (1 if none does; the call then fails in ensure_ws).  A caller's own batch size
// is kept as given.
int fit_static_S(const qst_handle* h, Geometry g, const qst_instance& in, int S, qst_path path, size_t base) {
  if (!h->static_ws || in.settings_per_batch > 0) return S;
  int lo = 1, hi = S;
  while (lo < hi) {
    const int mid = lo + (hi - lo + 1) / 2;
    set_grid(const_cast<qst_handle*>(h), g, mid);
    if (layout_ws(g, mid, path, false, base).total <= h->ws_bytes)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

qst_status run_instance(qst_handle* h, const RunSpec& rs, size_t ws_base = 0, size_t* ws_end = nullptr) {
  const qst_instance& in = *rs.in;
  const qst_path path = rs.path;
  Geometry g;
  qst_status st = make_geometry(h, in.n_qubits, in.rank, in.n_settings, path, g);
  if (st != QST_OK) return st;
  mark(g, in);
  const int S = rs.S_override > 0 ? batch_size(h, g, in, path, rs.S_override)
                                  : fit_static_S(h, g, in, batch_size(h, g, in, path, 0), path, ws_base);
  set_grid(h, g, S);
  const WsLayout L = layout_ws(g, S, path, false, ws_base);
  if (ws_end) *ws_end = L.total;
  st = ensure_ws(h, L.total);
  if (st != QST_OK) return st;
  unsigned char* ws = reinterpret_cast<unsigned char*>(h->ws);
  uint64_t* pc = reinterpret_cast<uint64_t*>(ws + L.pc);
  void* X = ws + L.X;
  void* W = ws + L.W;
  double* part = reinterpret_cast<double*>(ws + L.part);
  double* lvl1 = reinterpret_cast<double*>(ws + L.lvl1);
  double* sums = reinterpret_cast<double*>(ws + L.sums);
  hipStream_t s = h->stream;

  float* um = g.gen ? reinterpret_cast<float*>(ws + L.um) : nullptr;
  long long* cptr = g.sparse ? reinterpret_cast<long long*>(ws + L.cptr) : nullptr;
  prof_begin(h, PK_DECODE);
  if (g.gen)
    QST_HIP(qst::launch_decode_general(in.settings, g.B, g.n, in.unitaries, in.n_unitaries, um, pc, h->dflag, s));
  else
    QST_HIP(qst::launch_decode(in.settings, g.B, g.n, pc, h->dflag, s));
  if (g.sparse)
    QST_HIP(qst::launch_chunk_ptr(reinterpret_cast<const long long*>(in.freqs_rowptr), in.freqs_index,
                                  in.freqs_nnz, g.B, pass_path(path) ? 1 : (1 << g.n_hi), 1 << g.n_lo, cptr, s));
  prof_end(h);
  const bool want_loss = rs.grad_p == nullptr && rs.loss_kind != QST_LOSS_NONE;
  const long long nslots = nslots_of(g, path);

  qst::LoArgs la{};
  la.pc = pc;
  la.um = um;
  la.fidx = g.sparse ? in.freqs_index : nullptr;
  la.fchunk = cptr;
  la.fnnz = in.freqs_nnz;
  la.alpha = in.weights;
  la.freqs = in.freqs;
  la.grad_p = rs.grad_p;
  la.probs = rs.probs;
  la.pbase = in.probs_base;
  la.gneg = rs.gneg;
  la.part = (want_loss || rs.adjoint) ? part : nullptr;
  la.nslots = nslots;
  la.D = g.D;
  la.R = g.R;
  la.n = g.n;
  la.n_lo = g.n_lo;
  la.n_hi = g.n_hi;
  la.log_ta = g.n_lo - g.logv_lo;
  la.B = g.B;
  la.loss_kind = rs.grad_p ? 2 : (int)rs.loss_kind;
  la.eps = rs.eps;
  // the W layout only matters between the low stage and the adjoint top stage
  const bool reorder = g.n_hi > 0 && g.n_mid == 0 && !pass_path(path);
  la.w_up = (rs.adjoint && reorder) ? w_up_of(h, g, path) : 0;
  la.x_up = reorder ? x_up_of(h, g, path) : 0;

  for (int b0 = 0; b0 < g.B; b0 += S) {
    const int Sb = std::min(S, g.B - b0);
    la.b0 = b0;
    la.slot_base = (long long)(b0 / S) * g.grid_lo;
    la.nchunks = Sb << g.n_hi;
    if (pass_path(path)) {
      // groups of four qubits on the matrix cores (states of at least 2^8 amplitudes),
      // the remaining qubits one pass each
      const bool tiles = path != QST_PATH_PLAIN_F32 && g.D >= 256;
      const bool bf16 = path == QST_PATH_TILE_BF16;
      auto transform = [&](bool adj) -> qst_status {
        int bit = 0;
        if (tiles)
          for (; bit + 4 <= g.n; bit += 4)
            QST_HIP(qst::launch_tile_pass(X, Sb, g.R, g.D, bit, pc, b0, adj, bf16, s));
        for (; bit < g.n; ++bit) QST_HIP(qst::launch_plain_qubit(X, Sb, g.R, g.D, bit, pc, b0, adj, s));
        return QST_OK;
      };
      prof_begin(h, PK_OTHER);
      QST_HIP(qst::launch_plain_copy(in.atoms, X, Sb, g.R, g.D, s));
      st = transform(false);
      if (st != QST_OK) return st;
      QST_HIP(qst::launch_plain_point(la, X, Sb, s));
      if (rs.adjoint) {
        st = transform(true);
        if (st != QST_OK) return st;
        QST_HIP(qst::launch_plain_sum(X, Sb, g.R, g.D, rs.atom_grad, b0 == 0, s));
      }
      prof_end(h);
      continue;
    }
    // the middle pass of a three-pass schedule, in place on X (forward) or W (adjoint)
    auto mid_pass = [&](void* buf, bool adj) -> qst_status {
      qst::MidArgs ma{};
      ma.buf = buf;
      ma.pc = pc;
      ma.um = um;
      ma.D = g.D;
      ma.R = g.R;
      ma.n = g.n;
      ma.row_lo = g.n_lo;
      ma.rows = g.n_mid;
      ma.t = 14;
      ma.c = g.c_mid;
      ma.b0 = b0;
      ma.S = Sb;
      // the middle tiles are named by every bit outside them (R 2^(n - 14) tiles): the view
      // with those bits below the rows gives split_of that count
      Geometry gm = g;
      gm.n_lo = g.n - g.n_mid;
      gm.n_hi = g.n_mid;
      ma.nsplit = split_of(h, gm, g.c_mid, Sb);
      prof_begin(h, PK_MID);
      QST_HIP(qst::launch_stage_mid(g, ma, adj, s));
      prof_end(h);
      return QST_OK;
    };
    const Geometry gt = top_view(g);
    if (g.n_hi > 0) {
      qst::HiArgs ha{};
      ha.src = in.atoms;
      ha.dst = X;
      ha.pc = pc;
      ha.um = um;
      ha.D = g.D;
      ha.R = g.R;
      ha.n = g.n;
      ha.n_lo = gt.n_lo;
      ha.n_hi = gt.n_hi;
      ha.t = g.t;
      ha.c = g.c;
      ha.b0 = b0;
      ha.S = Sb;
      ha.first = 0;
      ha.nsplit = split_of(h, gt, g.c, Sb);
      ha.w_up = la.x_up;
      prof_begin(h, PK_HI_FWD);
      QST_HIP(qst::launch_stage_hi(gt, ha, false, s));
      prof_end(h);
      if (g.n_mid > 0) {
        st = mid_pass(X, false);
        if (st != QST_OK) return st;
      }
      la.src = X;
      la.src_set_stride = (long long)g.R * g.D;
    } else {
      la.src = in.atoms;
      la.src_set_stride = 0;
    }
    la.dst = W;
    prof_begin(h, PK_LO);
    if (g.lo2) {
      QST_HIP(qst::launch_stage_lo2(g, la, rs.adjoint, s));
    } else {
      qst::LoBatch lb{};
      lb.count = 1;
      lb.total = la.nchunks;
      lb.rmax = g.R;
      lb.begin[0] = 0;
      lb.begin[1] = la.nchunks;
      lb.a[0] = la;
      QST_HIP(qst::launch_stage_lo(g, lb, rs.adjoint, s));
    }
    prof_end(h);
    if (rs.adjoint) {
      if (g.n_hi > 0) {
        if (g.n_mid > 0) {
          st = mid_pass(W, true);
          if (st != QST_OK) return st;
        }
        qst::HiArgs hc{};
        hc.src = W;
        hc.dst = rs.atom_grad;
        hc.pc = pc;
        hc.um = um;
        hc.D = g.D;
        hc.R = g.R;
        hc.n = g.n;
        hc.n_lo = gt.n_lo;
        hc.n_hi = gt.n_hi;
        hc.t = g.t_adj;
        hc.c = g.c_adj;
        hc.b0 = b0;
        hc.S = Sb;
        hc.first = b0 == 0;
        hc.nsplit = std::min(g.split_adj, split_of(h, gt, g.c_adj, Sb));
        hc.part = ws + L.split;
        hc.w_up = la.w_up;
        prof_begin(h, PK_HI_ADJ);
        Geometry gc = gt;
        gc.t = g.t_adj;
        gc.c = g.c_adj;
        QST_HIP(qst::launch_stage_hi(gc, hc, true, s));
        if (hc.nsplit > 1)
          QST_HIP(qst::launch_sum_splits(g.elem, hc.part, hc.nsplit, (long long)g.R * g.D, rs.atom_grad, hc.first, s));
        prof_end(h);
      } else {
        prof_begin(h, PK_HI_ADJ);
        QST_HIP(qst::launch_sum_settings(g, W, Sb, rs.atom_grad, b0 == 0, s));
        prof_end(h);
      }
    }
  }
  prof_begin(h, PK_REDUCE);
  if (want_loss || rs.adjoint) {
    const int rows = rs.adjoint ? g.R + 1 : 1;
    QST_HIP(qst::launch_rowsum(part, rows, nslots, lvl1, G1, sums, s));
    if (!want_loss) {
      // rows 1..R only are meaningful; scatter without the loss
      QST_HIP(qst::launch_scatter_results(sums, rs.adjoint ? g.R : 0, nullptr, rs.adjoint ? rs.weight_grad : nullptr, s));
    } else {
      QST_HIP(qst::launch_scatter_results(sums, rs.adjoint ? g.R : 0, rs.loss, rs.adjoint ? rs.weight_grad : nullptr, s));
    }
  }
  if (rs.adjoint && rs.project_tangent) {
    QST_HIP(qst::launch_tangent(g.elem, in.atoms, rs.atom_grad, g.R, g.D, reinterpret_cast<double*>(ws + L.tan), G1, s));
  }
  prof_end(h);
  return QST_OK;
}

// ---------------------------------------------------------------- batches of small instances
// A call with several instances runs those whose state is one low-stage chunk (no
// high bits) and whose settings fit one batch as batches of up to kBatchMax
// instances with equal n: one launch per step for the whole batch (decode, fused
// low stage, sum over settings, reductions, tangent projection).
bool batchable(const Geometry& g, qst_path path) {
  return !pass_path(path) && g.n_hi == 0 && default_S(g) >= g.B;
}

struct BatchLayout {
  Geometry g;  // largest rank of the batch; grid of the fused launch
  std::vector<size_t> pc, W, part, cptr;
  size_t total = 0;
};

qst_status batch_layout(qst_handle* h, const std::vector<const RunSpec*>& rs, bool adjoint, size_t base,
                        BatchLayout& L) {
  const int n = rs[0]->in->n_qubits;
  const int elem = elem_of(rs[0]->path);
  int rmax = 1;
  long long total = 0;
  for (const RunSpec* r : rs) {
    rmax = std::max(rmax, (int)r->in->rank);
    total += r->in->n_settings;
  }
  qst_status st = make_geometry(h, n, rmax, (int)std::min<long long>(total, 1 << 30), rs[0]->path, L.g);
  if (st != QST_OK) return st;
  if (L.g.n_hi != 0) return set_err(h, QST_ERR_SHAPE, "batched instance does not fit one chunk");
  set_grid(h, L.g, (int)std::min<long long>(total, 1 << 30));
  size_t o = base;
  L.pc.clear();
  L.W.clear();
  L.part.clear();
  L.cptr.clear();
  for (const RunSpec* r : rs) {
    const qst_instance& in = *r->in;
    const size_t D = (size_t)1 << n;
    L.pc.push_back(o);
    o = al256(o + (size_t)in.n_settings * 8);
    L.W.push_back(o);
    if (adjoint) o = al256(o + (size_t)in.n_settings * in.rank * D * 2 * (L.g.h16 ? 2 : elem));
    L.part.push_back(o);
    o = al256(o + (size_t)(in.rank + 1) * L.g.grid_lo * 8);
    L.cptr.push_back(o);
    if (in.freqs_rowptr) o = al256(o + ((size_t)in.n_settings + 1) * 8);
  }
  L.total = o;
  return QST_OK;
}

qst_status run_batch(qst_handle* h, const std::vector<const RunSpec*>& rs) {
  const RunSpec& r0 = *rs[0];
  const bool adjoint = r0.adjoint;
  const bool want_loss = r0.grad_p == nullptr && r0.loss_kind != QST_LOSS_NONE;
  BatchLayout L;
  qst_status st = batch_layout(h, rs, adjoint, 0, L);
  if (st != QST_OK) return st;
  st = ensure_ws(h, L.total);
  if (st != QST_OK) return st;
  unsigned char* ws = reinterpret_cast<unsigned char*>(h->ws);
  hipStream_t s = h->stream;
  const int n = r0.in->n_qubits;
  const long long D = 1ll << n;
  const int count = (int)rs.size();

  qst::DecodeBatch db{};
  db.count = count;
  db.N = n;
  qst::LoBatch lb{};
  lb.count = count;
  lb.rmax = L.g.R;
  qst::SumBatch sb{};
  sb.count = count;
  sb.elem = L.g.elem;
  sb.h16 = L.g.h16 ? 1 : 0;
  qst::RowBatch rb{};
  rb.count = count;
  rb.rmax = L.g.R;
  rb.nslots = L.g.grid_lo;
  qst::TanBatch tb{};
  tb.count = count;
  tb.rmax = L.g.R;
  tb.elem = L.g.elem;
  int chunks = 0;
  long long elems = 0;
  for (int k = 0; k < count; ++k) {
    const RunSpec& r = *rs[k];
    const qst_instance& in = *r.in;
    uint64_t* pc = reinterpret_cast<uint64_t*>(ws + L.pc[k]);
    double* part = reinterpret_cast<double*>(ws + L.part[k]);
    long long* cptr = in.freqs_rowptr ? reinterpret_cast<long long*>(ws + L.cptr[k]) : nullptr;
    if (cptr)
      QST_HIP(qst::launch_chunk_ptr(reinterpret_cast<const long long*>(in.freqs_rowptr), in.freqs_index, in.freqs_nnz,
                                    in.n_settings, 1, 1 << n, cptr, s));
    db.begin[k] = chunks;
    db.settings[k] = in.settings;
    db.pc[k] = pc;
    qst::LoArgs& la = lb.a[k];
    la.src = in.atoms;
    la.src_set_stride = 0;
    la.dst = adjoint ? ws + L.W[k] : nullptr;
    la.pc = pc;
    la.alpha = in.weights;
    la.freqs = in.freqs;
    la.grad_p = r.grad_p;
    la.probs = r.probs;
    la.pbase = in.probs_base;
    la.fidx = cptr ? in.freqs_index : nullptr;
    la.fchunk = cptr;
    la.fnnz = in.freqs_nnz;
    la.gneg = nullptr;
    la.part = (want_loss || adjoint) ? part : nullptr;
    la.nslots = L.g.grid_lo;
    la.slot_base = 0;
    la.nchunks = in.n_settings;
    la.D = D;
    la.R = in.rank;
    la.n = n;
    la.n_lo = n;
    la.n_hi = 0;
    la.log_ta = L.g.n_lo - L.g.logv_lo;
    la.b0 = 0;
    la.B = in.n_settings;
    la.loss_kind = r.grad_p ? 2 : (int)r.loss_kind;
    la.eps = r.eps;
    lb.begin[k] = chunks;
    sb.begin[k] = elems;
    sb.W[k] = ws + L.W[k];
    sb.grad[k] = r.atom_grad;
    sb.RD[k] = (long long)in.rank * D;
    sb.S[k] = in.n_settings;
    rb.part[k] = part;
    rb.R[k] = in.rank;
    rb.loss[k] = want_loss ? r.loss : nullptr;
    rb.wgrad[k] = adjoint ? r.weight_grad : nullptr;
    tb.atoms[k] = in.atoms;
    tb.grad[k] = r.atom_grad;
    tb.R[k] = in.rank;
    tb.D[k] = D;
    chunks += in.n_settings;
    elems += (long long)in.rank * D;
  }
  db.begin[count] = lb.begin[count] = chunks;
  db.total = lb.total = chunks;
  sb.begin[count] = elems;
  sb.total = elems;

  prof_begin(h, PK_DECODE);
  QST_HIP(qst::launch_decode_batch(db, h->dflag, s));
  prof_end(h);
  prof_begin(h, PK_LO);
  QST_HIP(qst::launch_stage_lo(L.g, lb, adjoint, s));
  prof_end(h);
  if (adjoint) {
    prof_begin(h, PK_HI_ADJ);
    QST_HIP(qst::launch_sum_batch(sb, s));
    prof_end(h);
  }
  prof_begin(h, PK_REDUCE);
  if (want_loss || adjoint) QST_HIP(qst::launch_rowsum_batch(rb, s));
  if (adjoint && r0.project_tangent) QST_HIP(qst::launch_tangent_batch(tb, s));
  prof_end(h);
  return QST_OK;
}

// Runs the instances of one call: batches of small instances (equal n), the rest
// one by one.  `need` (optional) receives the workspace the call uses instead.
// ---------------------------------------------------------------- on-chip path (n = 11..14)
// Instances whose (setting, atom) vector fits one work-group run their whole rotation on
// chip (qst_onchip.hip): pass F forms p, the loss and 2^-k g per setting with the atoms
// looped, pass A recomputes each atom's rotation per setting and sums the adjoint over a
// slice of settings in registers.  No intermediate amplitudes cross HBM.
// FP32 Pauli settings with dense data and the library's own batch size: the kinds below apply.
bool dev_table_eligible(const RunSpec& r) {
  const qst_instance& in = *r.in;
  if (resolve(r.path) != QST_PATH_BUTTERFLY_F32) return false;
  return !in.unitaries && !in.freqs_rowptr && in.settings_per_batch <= 0;
}

bool oc_eligible(const RunSpec& r) {
  const qst_instance& in = *r.in;
  if (!dev_table_eligible(r) || in.n_qubits < 11 || in.n_qubits > 14) return false;
  // the outcome rows are read and written four values at a time
  auto a16 = [](const void* p) { return p == nullptr || aligned(p, 16); };
  return a16(in.freqs) && a16(in.probs_base) && a16(r.probs) && a16(r.grad_p) && a16(r.gneg) && a16(r.atom_grad) &&
         a16(in.atoms);
}

int env_int(const char* name, int dflt) {
  const char* e = std::getenv(name);
  return e ? std::atoi(e) : dflt;
}

// Experiment switches (environment, read once): QST_ONCHIP 0 never / 1 for every eligible
// instance (default: when R 2^n > 2^14), QST_FS 0 turns the fused slices off.
int env_onchip() {
  static const int v = env_int("QST_ONCHIP", -1);
  return v;
}
int env_fs() {
  static const int v = env_int("QST_FS", 1);
  return v;
}

// Kind of the device-table path an instance takes: 0 none, 1 atoms looped on chip (pass F and
// pass A), 2 fused slices (every atom of a setting in one work-group).
enum { TK_NONE = 0, TK_OC = 1, TK_FS = 2 };

// Order of precedence: the shape's choice (qst_plan_choice, autotune), the routing policy of
// the call (autotune of a multi-instance call), the environment switches, the default rule.
int table_kind(const qst_handle* h, const RunSpec& r) {
  if (!dev_table_eligible(r)) return TK_NONE;
  const qst_instance& in = *r.in;
  const bool fits = ((long long)in.rank << in.n_qubits) <= 16384;
  const bool fs_ok = fits && aligned(r.atom_grad, 8);
  if (const qst_choice* c = find_choice(h, in.n_qubits, in.rank, in.n_settings, resolve(r.path))) {
    if (c->kind == 0) return TK_NONE;
    if (c->kind == 1 && oc_eligible(r)) return TK_OC;
    if (c->kind == 2 && fs_ok) return TK_FS;
  }
  const int e = h->cur_policy.first >= 0 ? h->cur_policy.first : env_onchip();
  const int f = h->cur_policy.second >= 0 ? h->cur_policy.second : env_fs();
  if (oc_eligible(r) && (e == 1 || (e != 0 && !fits))) return TK_OC;
  if (fs_ok && f != 0) return TK_FS;
  return TK_NONE;
}

// Pass-A slicing of the atoms-looped kind: enough slices to give every resident work-group one
// item when the instance runs alone, no slice below QST_OC_SLICE_MIN settings (default 16),
// which bounds the slice partials written to HBM at 16 / S_min bytes per (setting, atom)
// amplitude.
// QST_GV_GROUPED=0 (read at every refactor call) sends the G v products through the staged
// path instead of the grouped low stage.
bool gv_grouped_on() {
  const char* e = std::getenv("QST_GV_GROUPED");
  return !(e && e[0] == '0');
}

int gv_occ(qst_handle* h) {
  if (h->gv_occupancy <= 0) h->gv_occupancy = qst::gv_blocks_per_cu(5);
  return h->gv_occupancy;
}

int env_oc_slice_min() {
  static const int v = [] {
    const int x = env_int("QST_OC_SLICE_MIN", 0);
    return x > 0 ? x : 16;
  }();
  return v;
}

// Items per resident work-group of the fused slices (QST_FS_ITEMS, default 1): the settings of
// a launch are cut into about that many slices per work-group slot, so a call of many small
// instances writes few partial gradients and a single one still fills the device; no slice
// has fewer than QST_FS_SLICE_MIN settings (default 4).
int env_fs_items() {
  static const int v = [] {
    const int x = env_int("QST_FS_ITEMS", 0);
    return x > 0 ? x : 1;
  }();
  return v;
}
int env_fs_slice_min() {
  static const int v = [] {
    const int x = env_int("QST_FS_SLICE_MIN", 0);
    return x > 0 ? x : 4;
  }();
  return v;
}

// Values per thread of the atoms-looped passes: QST_OC_LOGV (environment, read once) if it names
// a supported shape, else 2^5.
int oc_logv(const qst_handle* h, const RunSpec& r) {
  static const int v = env_int("QST_OC_LOGV", 0);
  const int n = r.in->n_qubits;
  if (const qst_choice* c = find_choice(h, n, r.in->rank, r.in->n_settings, resolve(r.path)))
    if (qst::oc_shape_ok(n, c->values_per_thread_log2)) return c->values_per_thread_log2;
  return qst::oc_shape_ok(n, v) ? v : 5;
}

int oc_occ(qst_handle* h, int n, int logv, bool adj) {
  const auto key = std::make_pair(n * 16 + logv, adj ? 1 : 0);
  auto it = h->oc_occupancy.find(key);
  if (it == h->oc_occupancy.end()) it = h->oc_occupancy.emplace(key, qst::oc_blocks_per_cu(n, logv, adj)).first;
  return it->second;
}

int fs_occ(qst_handle* h, int n, int RM, bool adj) {
  const auto key = std::make_pair(1000 + n * 64 + RM, adj ? 1 : 0);
  auto it = h->oc_occupancy.find(key);
  if (it == h->oc_occupancy.end()) it = h->oc_occupancy.emplace(key, qst::fs_blocks_per_cu(n, adj, RM)).first;
  return it->second;
}

// The device-table path: one instance table in the workspace, then per (kind, n) one launch
// of each pass over all instances of that class, then one launch each of the slice sums,
// the loss and weight-gradient sums and the tangent projection.
qst_status run_table(qst_handle* h, std::vector<const RunSpec*> rs, size_t* need) {
  // classes (kind, n) in order, larger instances first inside a class
  std::stable_sort(rs.begin(), rs.end(), [h](const RunSpec* a, const RunSpec* b) {
    const int ka = table_kind(h, *a), kb = table_kind(h, *b);
    if (ka != kb) return ka < kb;
    if (a->in->n_qubits != b->in->n_qubits) return a->in->n_qubits > b->in->n_qubits;
    const int la = ka == TK_OC ? oc_logv(h, *a) : 0, lb = kb == TK_OC ? oc_logv(h, *b) : 0;
    if (la != lb) return la < lb;
    return (long long)a->in->n_settings * a->in->rank > (long long)b->in->n_settings * b->in->rank;
  });
  const int count = (int)rs.size();
  struct Group {
    int kind, n, logv, RM, k0, k1, itemsF, itemsA;
    long long settings;
  };
  std::vector<Group> groups;
  for (int k = 0; k < count; ++k) {
    const int kind = table_kind(h, *rs[k]);
    const int n = rs[k]->in->n_qubits;
    const int logv = kind == TK_OC ? oc_logv(h, *rs[k]) : 5;
    if (groups.empty() || groups.back().kind != kind || groups.back().n != n || groups.back().logv != logv)
      groups.push_back(Group{kind, n, logv, 1, k, k, 0, 0, 0});
    Group& gr = groups.back();
    gr.k1 = k + 1;
    gr.RM = std::max(gr.RM, (int)rs[k]->in->rank);
    gr.settings += rs[k]->in->n_settings;
  }
  std::vector<qst::OcInst> tab(count);
  size_t o = al256((size_t)count * sizeof(qst::OcInst));
  std::vector<size_t> off_pc(count), off_G(count), off_P(count), off_part(count);
  int rmax = 1, sum_blocks = 0, dec_blocks = 0;
  bool any_rows = false, any_tan = false;
  for (Group& gr : groups) {
    const bool adj_any = rs[gr.k0]->adjoint;
    // fused slices: settings per slice from the launch's total (about env_fs_items() per slot)
    int fs_slice = 1;
    if (gr.kind == TK_FS) {
      const long long slots = (long long)h->num_cu * fs_occ(h, gr.n, gr.RM, adj_any) * env_fs_items();
      fs_slice = (int)std::max<long long>(env_fs_slice_min(), (gr.settings + slots - 1) / slots);
    }
    for (int k = gr.k0; k < gr.k1; ++k) {
      const RunSpec& r = *rs[k];
      const qst_instance& in = *r.in;
      qst::OcInst& a = tab[k];
      a = qst::OcInst{};
      const int n = in.n_qubits, R = in.rank, B = in.n_settings;
      const long long D = 1ll << n;
      a.n = n;
      a.R = R;
      a.B = B;
      a.eps = r.eps;
      a.loss_kind = r.grad_p ? 2 : (int)r.loss_kind;
      const bool fpass = gr.kind == TK_OC && r.grad_p == nullptr;  // the caller's dL/dp replaces pass F
      int nF = 0;
      if (gr.kind == TK_OC) {
        const int vpw = qst::oc_threads_of(n, gr.logv) >> (n - gr.logv);
        a.ntile = (R + vpw - 1) / vpw;
        a.sF = vpw;
        nF = fpass ? (B + a.sF - 1) / a.sF : 0;
        if (r.adjoint) {
          const int resident = h->num_cu * oc_occ(h, n, gr.logv, true);
          const int fill = (resident + a.ntile - 1) / a.ntile;
          const int most = std::max(1, B / env_oc_slice_min());
          const int nA0 = std::max(1, std::min(fill, most));
          a.sA = std::max((B + nA0 - 1) / nA0, a.sF);
          a.nA = (B + a.sA - 1) / a.sA;
        } else {
          a.sA = B;
          a.nA = 0;
        }
      } else {
        a.ntile = 1;
        a.sF = 1;
        a.sA = fs_slice;
        a.nA = (B + fs_slice - 1) / fs_slice;
      }
      a.nslots = std::max(nF, std::max(a.nA, 1));
      a.itemF0 = gr.itemsF;
      gr.itemsF += nF;
      a.itemA0 = gr.itemsA;
      if (gr.kind == TK_FS || r.adjoint) gr.itemsA += a.nA * a.ntile;
      a.tangent = r.adjoint && r.project_tangent ? 1 : 0;
      rmax = std::max(rmax, R);
      a.loss = (r.grad_p == nullptr && r.loss_kind != QST_LOSS_NONE) ? r.loss : nullptr;
      a.wgrad = r.adjoint ? r.weight_grad : nullptr;
      any_rows |= a.loss != nullptr || a.wgrad != nullptr;
      any_tan |= a.tangent != 0;
      off_pc[k] = o;
      o = al256(o + (size_t)B * 8);
      off_G[k] = o;
      if (r.adjoint && fpass) o = al256(o + (size_t)B * D * 4);
      off_P[k] = o;
      if (r.adjoint && a.nA > 1) o = al256(o + (size_t)a.nA * R * D * 8);
      off_part[k] = o;
      o = al256(o + (size_t)(R + 1) * a.nslots * 8);
      a.sumB0 = sum_blocks;
      if (r.adjoint && a.nA > 1) sum_blocks += (int)(((long long)R * D + 31) / 32);
      a.decB0 = dec_blocks;
      dec_blocks += (B + 255) / 256;
    }
  }
  if (need) {
    *need = std::max(*need, o);
    return QST_OK;
  }
  qst_status st = ensure_ws(h, o);
  if (st != QST_OK) return st;
  unsigned char* ws = reinterpret_cast<unsigned char*>(h->ws);
  hipStream_t s = h->stream;
  qst::OcInst* dtab = reinterpret_cast<qst::OcInst*>(ws);
  for (int k = 0; k < count; ++k) {
    const RunSpec& r = *rs[k];
    const qst_instance& in = *r.in;
    qst::OcInst& a = tab[k];
    const bool oc = table_kind(h, r) == TK_OC;
    a.atoms = in.atoms;
    a.alpha = in.weights;
    a.pc = reinterpret_cast<const uint64_t*>(ws + off_pc[k]);
    a.pc_out = reinterpret_cast<uint64_t*>(ws + off_pc[k]);
    a.settings = in.settings;
    a.freqs = r.grad_p ? nullptr : in.freqs;
    a.grad_p = reinterpret_cast<const float*>(r.grad_p);
    a.pbase = reinterpret_cast<const float*>(in.probs_base);
    a.probs = reinterpret_cast<float*>(r.probs);
    a.gneg = reinterpret_cast<float*>(r.gneg);
    a.G = (oc && r.adjoint && r.grad_p == nullptr) ? reinterpret_cast<float*>(ws + off_G[k]) : nullptr;
    a.P = (r.adjoint && a.nA > 1) ? reinterpret_cast<float2*>(ws + off_P[k]) : nullptr;
    a.grad = r.adjoint ? reinterpret_cast<float2*>(r.atom_grad) : nullptr;
    a.part = reinterpret_cast<double*>(ws + off_part[k]);
  }
  prof_begin(h, PK_DECODE);
  for (int c0 = 0; c0 < count; c0 += qst::kOcChunk) {
    qst::OcChunk ch{};
    ch.first = c0;
    ch.count = std::min(qst::kOcChunk, count - c0);
    for (int i = 0; i < ch.count; ++i) ch.a[i] = tab[c0 + i];
    QST_HIP(qst::launch_oc_stage(ch, dtab, s));
  }
  QST_HIP(qst::launch_oc_decode(dtab, count, dec_blocks, h->dflag, s));
  prof_end(h);
  // The classes touch disjoint instances (their own outputs and workspace rows) and read
  // only the decoded table, so with more than one class each runs on a side stream forked
  // from s after the decode; s waits for all of them before the sums.  With stage timing
  // on, everything stays on s.
  const bool fork = groups.size() > 1 && h->side_ok && !h->prof;
  bool used[qst_handle::kSide] = {};
  if (fork) QST_HIP(hipEventRecord(h->fork_ev, s));
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const Group& gr = groups[gi];
    const bool adj = rs[gr.k0]->adjoint;
    hipStream_t gs = s;
    if (fork) {
      const int j = (int)(gi % qst_handle::kSide);
      gs = h->side[j];
      if (!used[j]) {
        QST_HIP(hipStreamWaitEvent(gs, h->fork_ev, 0));
        used[j] = true;
      }
    }
    if (gr.kind == TK_FS) {
      const int grid =
          (int)std::min<long long>(gr.itemsA, (long long)h->num_cu * fs_occ(h, gr.n, gr.RM, adj));
      prof_begin(h, PK_LO);
      QST_HIP(qst::launch_fs_pass(gr.n, adj, dtab, gr.k0, gr.k1, gr.itemsA, gr.RM, grid, gs));
      prof_end(h);
      continue;
    }
    if (gr.itemsF > 0) {
      const int grid = (int)std::min<long long>(gr.itemsF, (long long)h->num_cu * oc_occ(h, gr.n, gr.logv, false));
      prof_begin(h, PK_HI_FWD);
      QST_HIP(qst::launch_oc_pass(gr.n, gr.logv, false, dtab, gr.k0, gr.k1, gr.itemsF, grid, gs));
      prof_end(h);
    }
    if (gr.itemsA > 0) {
      const int grid = (int)std::min<long long>(gr.itemsA, (long long)h->num_cu * oc_occ(h, gr.n, gr.logv, true));
      prof_begin(h, PK_LO);
      QST_HIP(qst::launch_oc_pass(gr.n, gr.logv, true, dtab, gr.k0, gr.k1, gr.itemsA, grid, gs));
      prof_end(h);
    }
  }
  if (fork)
    for (int j = 0; j < qst_handle::kSide; ++j)
      if (used[j]) {
        QST_HIP(hipEventRecord(h->join_ev[j], h->side[j]));
        QST_HIP(hipStreamWaitEvent(s, h->join_ev[j], 0));
      }
  if (sum_blocks > 0 || any_rows || any_tan) {
    prof_begin(h, PK_REDUCE);
    QST_HIP(qst::launch_oc_finish(dtab, count, sum_blocks, rmax, any_rows, any_tan, s));
    prof_end(h);
  }
  return QST_OK;
}

// Signature of a multi-instance call (FNV-1a over every instance's n, R, B and path, in order):
// the key of its routing policy.
uint64_t call_signature(const std::vector<RunSpec>& specs) {
  uint64_t x = 1469598103934665603ull;
  auto mix = [&](uint64_t v) {
    x ^= v;
    x *= 1099511628211ull;
  };
  for (const RunSpec& r : specs) {
    mix((uint64_t)r.in->n_qubits);
    mix((uint64_t)r.in->rank);
    mix((uint64_t)r.in->n_settings);
    mix((uint64_t)resolve(r.path));
  }
  return x;
}

qst_status run_call_inner(qst_handle* h, const std::vector<RunSpec>& specs, size_t* need);

qst_status run_call(qst_handle* h, const std::vector<RunSpec>& specs, size_t* need = nullptr) {
  // the routing policy kept for this call's shapes (several instances) applies while it runs
  const std::pair<int, int> saved = h->cur_policy;
  if (specs.size() > 1 && !h->policies.empty()) {
    auto it = h->policies.find(call_signature(specs));
    if (it != h->policies.end()) h->cur_policy = it->second;
  }
  const qst_status st = run_call_inner(h, specs, need);
  h->cur_policy = saved;
  return st;
}

qst_status run_call_inner(qst_handle* h, const std::vector<RunSpec>& specs, size_t* need) {
  std::map<int, std::vector<const RunSpec*>> groups;
  std::vector<const RunSpec*> single;
  std::vector<const RunSpec*> onchip;
  for (const RunSpec& r : specs)
    if (table_kind(h, r) != TK_NONE) onchip.push_back(&r);
  if (!onchip.empty() && h->static_ws) {
    // without allocation the table path's buffers must fit the static scratch, else the staged path runs
    size_t oc_need = 0;
    qst_status st = run_table(h, onchip, &oc_need);
    if (st != QST_OK) return st;
    if (oc_need > h->ws_bytes) onchip.clear();
  }
  if (!onchip.empty()) {
    qst_status st = run_table(h, onchip, need);
    if (st != QST_OK) return st;
  }
  for (const RunSpec& r : specs) {
    if (std::find(onchip.begin(), onchip.end(), &r) != onchip.end()) continue;
    Geometry g;
    qst_status st = make_geometry(h, r.in->n_qubits, r.in->rank, r.in->n_settings, r.path, g);
    if (st != QST_OK) return st;
    if (specs.size() > 1 && batchable(g, r.path) && r.in->settings_per_batch <= 0 && !r.in->unitaries)
      groups[r.in->n_qubits].push_back(&r);
    else
      single.push_back(&r);
  }
  for (auto& kv : groups) {
    const std::vector<const RunSpec*>& v = kv.second;
    for (size_t b0 = 0; b0 < v.size(); b0 += qst::kBatchMax) {
      std::vector<const RunSpec*> part(v.begin() + b0, v.begin() + std::min(v.size(), b0 + qst::kBatchMax));
      if (part.size() == 1) {
        single.push_back(part[0]);
        continue;
      }
      if (h->static_ws) {
        // a batch whose buffers do not fit the static scratch runs one instance at a time
        BatchLayout L;
        qst_status st = batch_layout(h, part, part[0]->adjoint, 0, L);
        if (st != QST_OK) return st;
        if (L.total > h->ws_bytes) {
          single.insert(single.end(), part.begin(), part.end());
          continue;
        }
      }
      if (need) {
        BatchLayout L;
        qst_status st = batch_layout(h, part, part[0]->adjoint, 0, L);
        if (st != QST_OK) return st;
        *need = std::max(*need, L.total);
        continue;
      }
      qst_status st = run_batch(h, part);
      if (st != QST_OK) return st;
    }
  }
  for (const RunSpec* r : single) {
    if (need) {
      Geometry g;
      qst_status st = make_geometry(h, r->in->n_qubits, r->in->rank, r->in->n_settings, r->path, g);
      if (st != QST_OK) return st;
      mark(g, *r->in);
      const int S = fit_static_S(h, g, *r->in, batch_size(h, g, *r->in, r->path, 0), r->path, 0);
      set_grid(h, g, S);
      *need = std::max(*need, layout_ws(g, S, r->path, false).total);
      continue;
    }
    qst_status st = run_instance(h, *r);
    if (st != QST_OK) return st;
  }
  return QST_OK;
}

// ---------------------------------------------------------------- small dense helpers (host FP64)
// Cyclic Jacobi eigenvalue iteration for a real symmetric k x k matrix (row-major).
// Returns eigenvalues in w and eigenvectors as columns of V.
void jacobi_eigh(std::vector<double> A, int k, std::vector<double>& w, std::vector<double>& V) {
  V.assign((size_t)k * k, 0.0);
  for (int i = 0; i < k; ++i) V[(size_t)i * k + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) {
        const double a = A[(size_t)i * k + j];
        tot += a * a;
        if (i != j) off += a * a;
      }
    if (off <= 1e-30 * std::max(tot, 1e-300)) break;
    for (int p = 0; p < k - 1; ++p)
      for (int q = p + 1; q < k; ++q) {
        const double apq = A[(size_t)p * k + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double app = A[(size_t)p * k + p], aqq = A[(size_t)q * k + q];
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        for (int r = 0; r < k; ++r) {  // A <- J^T A J
          const double arp = A[(size_t)r * k + p], arq = A[(size_t)r * k + q];
          A[(size_t)r * k + p] = c * arp - sn * arq;
          A[(size_t)r * k + q] = sn * arp + c * arq;
        }
        for (int r = 0; r < k; ++r) {
          const double apr = A[(size_t)p * k + r], aqr = A[(size_t)q * k + r];
          A[(size_t)p * k + r] = c * apr - sn * aqr;
          A[(size_t)q * k + r] = sn * apr + c * aqr;
        }
        for (int r = 0; r < k; ++r) {
          const double vrp = V[(size_t)r * k + p], vrq = V[(size_t)r * k + q];
          V[(size_t)r * k + p] = c * vrp - sn * vrq;
          V[(size_t)r * k + q] = sn * vrp + c * vrq;
        }
      }
  }
  w.resize(k);
  for (int i = 0; i < k; ++i) w[i] = A[(size_t)i * k + i];
}

// Euclidean projection onto the simplex (sort-based), FP64.
std::vector<double> proj_simplex(const std::vector<double>& v) {
  std::vector<double> u = v;
  std::sort(u.begin(), u.end(), [](double a, double b) { return a > b; });
  double css = 0.0, theta = 0.0;
  for (size_t j = 0; j < u.size(); ++j) {
    css += u[j];
    const double t = (css - 1.0) / (double)(j + 1);
    if (u[j] - t > 0) theta = t;
  }
  std::vector<double> out(v.size());
  for (size_t i = 0; i < v.size(); ++i) out[i] = std::max(v[i] - theta, 0.0);
  return out;
}

}  // namespace

// Device address of `scratch` on `device` (which must be current): looked up once per device
// and kept until the process ends.
static std::mutex g_scratch_mu;
static std::map<int, void*> g_scratch_addr;

static hipError_t scratch_address(int device, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_addr.find(device);
  if (it != g_scratch_addr.end()) {
    *out = it->second;
    return hipSuccess;
  }
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || p == nullptr) return e != hipSuccess ? e : hipErrorInvalidSymbol;
  g_scratch_addr.emplace(device, p);
  *out = p;
  return hipSuccess;
}

// Internal access for the host-orchestrated iteration (qst_solve.hip); not exported.
#define QST_HIDDEN __attribute__((visibility("hidden")))
QST_HIDDEN hipStream_t qst_host_stream(qst_handle* h) { return h->stream; }
QST_HIDDEN qst_status qst_host_error(qst_handle* h, qst_status s, const std::string& msg) { return set_err(h, s, msg); }
QST_HIDDEN int qst_host_device(const qst_handle* h) { return h->device; }

// ==================================================================== C ABI
extern "C" {

const char* qst_status_string(qst_status s) {
  switch (s) {
    case QST_OK: return "ok";
    case QST_ERR_INVALID_ARG: return "invalid argument";
    case QST_ERR_SHAPE: return "unsupported shape";
    case QST_ERR_ALIGN: return "misaligned pointer";
    case QST_ERR_UNSUPPORTED: return "unsupported request";
    case QST_ERR_DEVICE: return "HIP runtime error";
    case QST_ERR_OOM: return "out of device memory";
    case QST_ERR_NUMERIC: return "numeric fault flagged by a kernel";
    case QST_ERR_CAPTURE: return "allocation requested during stream capture";
  }
  return "unknown status";
}

qst_status qst_profile_enable(qst_handle* h, int enable) {
  if (!h) return QST_ERR_INVALID_ARG;
  if (h->device < 0) return set_err(h, QST_ERR_UNSUPPORTED, "validation-only handle");
  if (enable && capturing(h->stream)) return set_err(h, QST_ERR_CAPTURE, "enable profiling outside capture");
  h->prof = enable != 0;
  return QST_OK;
}

qst_status qst_profile_read(qst_handle* h, int kind, int64_t* launches, double* total_ms, int reset) {
  if (!h || !launches || !total_ms) return QST_ERR_INVALID_ARG;
  if (kind < 0 || kind >= kProfKinds) return set_err(h, QST_ERR_INVALID_ARG, "kind must be in 0..7");
  *launches = 0;
  *total_ms = 0.0;
  if (h->device < 0) return QST_OK;
  if (hipStreamSynchronize(h->stream) != hipSuccess) return set_err(h, QST_ERR_DEVICE, "stream synchronise failed");
  for (const auto& m : h->marks) {
    if (m.kind != kind) continue;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, m.a, m.b) == hipSuccess) {
      *launches += 1;
      *total_ms += ms;
    }
  }
  if (reset) {
    h->marks.clear();
    h->ev_next = 0;
  }
  return QST_OK;
}

const char* qst_build_info(void) { return "qst gfx950 staged-butterfly/tile v1"; }

const char* qst_last_error(const qst_handle* h) { return h ? h->last_error.c_str() : "null handle"; }

qst_status qst_create(int device, void* hip_stream, qst_handle** out) {
  if (!out) return QST_ERR_INVALID_ARG;
  *out = nullptr;
  if (device == -1) {  // validation-only handle: argument checks run, nothing is enqueued
    qst_handle* h = new qst_handle();
    h->device = -1;
    *out = h;
    return QST_OK;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return QST_ERR_DEVICE;
  if (device < 0 || device >= ndev) return QST_ERR_INVALID_ARG;
  if (hipSetDevice(device) != hipSuccess) return QST_ERR_DEVICE;
  qst_handle* h = new qst_handle();
  h->device = device;
  h->stream = reinterpret_cast<hipStream_t>(hip_stream);
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
      if (prop.multiProcessorCount > 0) h->num_cu = prop.multiProcessorCount;
      h->arch = prop.gcnArchName;
    }
  }
  if (hipMalloc(&h->dflag, sizeof(int)) != hipSuccess || hipHostMalloc(&h->hflag, sizeof(int)) != hipSuccess ||
      hipEventCreateWithFlags(&h->flag_ev, hipEventDisableTiming) != hipSuccess) {
    delete h;
    return QST_ERR_DEVICE;
  }
  *h->hflag = 0;
  if (hipMemset(h->dflag, 0, sizeof(int)) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    (void)hipFree(h->dflag);
    (void)hipHostFree(h->hflag);
    (void)hipEventDestroy(h->flag_ev);
    delete h;
    return QST_ERR_DEVICE;
  }
  if (scratch_address(device, &h->static_scratch) != hipSuccess) h->static_scratch = nullptr;
  // side streams for the classes of multi-instance calls; without them the classes run one
  // after another on the handle's stream
  h->side_ok = hipEventCreateWithFlags(&h->fork_ev, hipEventDisableTiming) == hipSuccess;
  for (int i = 0; i < qst_handle::kSide && h->side_ok; ++i)
    h->side_ok = hipStreamCreateWithFlags(&h->side[i], hipStreamNonBlocking) == hipSuccess &&
                 hipEventCreateWithFlags(&h->join_ev[i], hipEventDisableTiming) == hipSuccess;
  *out = h;
  return QST_OK;
}

qst_status qst_destroy(qst_handle* h) {
  if (!h) return QST_ERR_INVALID_ARG;
  if (h->device < 0) {
    delete h;
    return QST_OK;
  }
  // teardown: every release is attempted; their statuses are not reported
  (void)hipSetDevice(h->device);
  (void)hipStreamSynchronize(h->stream);
  if (h->ws) (void)hipFree(h->ws);
  for (void* p : h->retired) (void)hipFree(p);
  if (h->dflag) (void)hipFree(h->dflag);
  if (h->hflag) (void)hipHostFree(h->hflag);
  if (h->flag_ev) (void)hipEventDestroy(h->flag_ev);
  for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
  for (int i = 0; i < qst_handle::kSide; ++i) {
    if (h->side[i]) (void)hipStreamDestroy(h->side[i]);
    if (h->join_ev[i]) (void)hipEventDestroy(h->join_ev[i]);
  }
  if (h->fork_ev) (void)hipEventDestroy(h->fork_ev);
  delete h;
  return QST_OK;
}

qst_status qst_set_stream(qst_handle* h, void* hip_stream) {
  if (!h) return QST_ERR_INVALID_ARG;
  h->stream = reinterpret_cast<hipStream_t>(hip_stream);
  return QST_OK;
}

static qst_status common_checks(qst_handle* h, const qst_instance* inst, int n_inst, qst_path path) {
  if (!h) return QST_ERR_INVALID_ARG;
  h->last_error.clear();
  if (!inst || n_inst < 1) return set_err(h, QST_ERR_INVALID_ARG, "no instances");
  if (!path_valid(path)) return set_err(h, QST_ERR_INVALID_ARG, "bad path");
  if (h->device < 0) return QST_OK;
  if (hipSetDevice(h->device) != hipSuccess) return set_err(h, QST_ERR_DEVICE, "hipSetDevice failed");
  return check_flag(h);
}

// After validation: a validation-only handle stops here.
static qst_status device_gate(qst_handle* h) {
  if (h->device < 0) return set_err(h, QST_ERR_UNSUPPORTED, "validation-only handle (device -1): arguments are valid");
  return QST_OK;
}

// ---------------------------------------------------------------- autotuning
// Candidates are timed as whole backward calls (CE loss, weight and atom gradients) on the
// handle's stream: one warm-up, then the median of three event-timed runs.  Their outputs go to
// the end of the workspace, which is grown once to hold the largest candidate.
static std::mutex g_tune_mu;
static std::map<std::pair<std::string, std::tuple<int, int, int, int>>, qst_choice> g_choice_cache;
static std::map<std::pair<std::string, uint64_t>, std::pair<int, int>> g_policy_cache;

struct Timer {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  Timer() {
    if (hipEventCreate(&e0) != hipSuccess) e0 = nullptr;
    if (hipEventCreate(&e1) != hipSuccess) e1 = nullptr;
  }
  ~Timer() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
};

// Median time (ms) of the call, or a negative value when it fails (the candidate is then skipped).
static double time_call(qst_handle* h, const std::vector<RunSpec>& specs, Timer& tm) {
  if (!tm.e0 || !tm.e1 || run_call(h, specs) != QST_OK) return -1.0;
  std::vector<float> ts;
  for (int rep = 0; rep < 3; ++rep) {
    if (hipEventRecord(tm.e0, h->stream) != hipSuccess) return -1.0;
    if (run_call(h, specs) != QST_OK) return -1.0;
    if (hipEventRecord(tm.e1, h->stream) != hipSuccess || hipEventSynchronize(tm.e1) != hipSuccess) return -1.0;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, tm.e0, tm.e1) != hipSuccess) return -1.0;
    ts.push_back(ms);
  }
  std::sort(ts.begin(), ts.end());
  return ts[1];
}

// Backward specs over `ins` with their outputs in the workspace after `base` (grown as needed).
static qst_status tune_specs(qst_handle* h, const std::vector<qst_instance>& ins, qst_path path, size_t base,
                             std::vector<RunSpec>& specs) {
  size_t out = 0;
  for (const qst_instance& in : ins)
    out += al256((size_t)in.rank * ((size_t)1 << in.n_qubits) * 2 * elem_of(path)) + al256((size_t)in.rank * 8 + 8);
  qst_status st = ensure_ws(h, base + out);
  if (st != QST_OK) return st;
  unsigned char* o = reinterpret_cast<unsigned char*>(h->ws) + base;
  specs.assign(ins.size(), RunSpec{});
  for (size_t k = 0; k < ins.size(); ++k) {
    RunSpec& r = specs[k];
    r.in = &ins[k];
    r.path = path;
    r.loss_kind = ins[k].freqs ? QST_LOSS_CE : QST_LOSS_NONE;
    r.eps = 1e-8;
    r.adjoint = true;
    r.atom_grad = o;
    o += al256((size_t)ins[k].rank * ((size_t)1 << ins[k].n_qubits) * 2 * elem_of(path));
    r.weight_grad = reinterpret_cast<double*>(o);
    r.loss = r.weight_grad + ins[k].rank;
    o += al256((size_t)ins[k].rank * 8 + 8);
  }
  return QST_OK;
}

// One instance: its kernels (staged / atoms looped / fused slices), batch size and tile bits,
// timed on a slice of at most 256 of its settings.
static qst_status tune_shape(qst_handle* h, const qst_instance& in0, qst_path path) {
  const auto key = shape_key(in0.n_qubits, in0.rank, in0.n_settings, path);
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_choice_cache.find(std::make_pair(h->arch, key));
    if (it != g_choice_cache.end()) {
      h->choices[key] = it->second;
      return QST_OK;
    }
  }
  if (!in0.freqs) return QST_OK;  // the timing runs the CE backward
  std::vector<qst_instance> ins(1, in0);
  ins[0].n_settings = std::min(in0.n_settings, 256);
  ins[0].settings_per_batch = 0;
  const int n = in0.n_qubits, R = in0.rank;
  Geometry g;
  const bool staged_ok = make_geometry(h, n, R, in0.n_settings, path, g) == QST_OK;
  h->last_error.clear();
  // candidate list: (kind, S, t_fwd, t_adj, logv)
  std::vector<qst_choice> cands;
  auto cand = [&](int kind, int S, int tf, int ta, int lv) {
    qst_choice c{};
    c.kind = kind;
    c.settings_per_batch = S;
    c.tile_bits_fwd = tf;
    c.tile_bits_adj = ta;
    c.values_per_thread_log2 = lv;
    cands.push_back(c);
  };
  cand(-1, 0, 0, 0, 0);  // the default
  RunSpec probe{};
  probe.in = &ins[0];
  probe.path = path;
  probe.atom_grad = h->ws;  // alignment probe only (the workspace base is 256-byte aligned)
  if (staged_ok) cand(0, 0, 0, 0, 0);
  if (oc_eligible(probe)) {
    cand(1, 0, 0, 0, 5);
    if (n == 13 || n == 14) cand(1, 0, 0, 0, 4);
  }
  if (((long long)R << n) <= 16384 && dev_table_eligible(probe)) cand(2, 0, 0, 0, 0);
  if (staged_ok && g.n_hi > 0) {
    const size_t per = (size_t)R * ((size_t)1 << n) * 2 * elem_of(path);
    for (int S : {16, 32, 64, 128})
      if (S <= ins[0].n_settings && (size_t)S * per <= (16ull << 30)) cand(0, S, 0, 0, 0);
    for (int t : {13, 12})
      if (t < 14 && g.n_hi <= (t == 13 ? 3 : 2) && t - g.n_hi <= g.n_lo) {
        cand(0, 0, t, 0, 0);
        cand(0, 0, 0, t, 0);
      }
    // the orders of X and W between the tile stages and the low stage (two passes)
    if (g.n_mid == 0) {
      for (int wb : {5, 6, g.n_lo})
        if (wb >= g.c_adj && wb <= g.n_lo && (wb != g.n_lo || wb > 6)) {
          cand(0, 0, 0, 0, 0);
          cands.back().w_row_bits = wb;
        }
      for (int xb : {6, g.n_lo})
        if (xb >= g.c && xb <= g.n_lo && (xb != g.n_lo || xb > 6)) {
          cand(0, 0, 0, 0, 0);
          cands.back().x_row_bits = xb;
        }
    }
  }
  // workspace: the largest candidate, then the outputs
  size_t need = 0;
  std::vector<RunSpec> specs;
  qst_status st = tune_specs(h, ins, path, 0, specs);
  if (st != QST_OK) return st;
  for (const qst_choice& c : cands) {
    h->choices[key] = c;
    size_t nd = 0;
    if (run_call(h, specs, &nd) == QST_OK) need = std::max(need, nd);
  }
  h->last_error.clear();
  st = tune_specs(h, ins, path, al256(need), specs);
  if (st != QST_OK) return st;
  Timer tm;
  double best = -1.0, dflt = -1.0;
  qst_choice chosen{};
  chosen.kind = -1;
  for (const qst_choice& c : cands) {
    h->choices[key] = c;
    const double ms = time_call(h, specs, tm);
    h->last_error.clear();
    if (ms < 0) continue;
    if (c.kind == -1) dflt = ms;
    if (best < 0 || ms < best) {
      best = ms;
      chosen = c;
    }
  }
  if (hipStreamSynchronize(h->stream) != hipSuccess) return set_err(h, QST_ERR_DEVICE, "autotune synchronise failed");
  chosen.tuned = 1;
  chosen.best_ms = best;
  chosen.default_ms = dflt;
  h->choices[key] = chosen;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_choice_cache[std::make_pair(h->arch, key)] = chosen;
  return QST_OK;
}

// Several instances: the routing of the whole call (atoms looped for every eligible instance or
// only where the atoms do not fit one work-group; fused slices on or off), timed on the call.
static qst_status tune_policy(qst_handle* h, const qst_instance* inst, int n_inst, qst_path path) {
  std::vector<qst_instance> ins(inst, inst + n_inst);
  for (const qst_instance& in : ins)
    if (!in.freqs) return QST_OK;
  std::vector<RunSpec> specs;
  qst_status st = tune_specs(h, ins, path, 0, specs);
  if (st != QST_OK) return st;
  const uint64_t sig = call_signature(specs);
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_policy_cache.find(std::make_pair(h->arch, sig));
    if (it != g_policy_cache.end()) {
      h->policies[sig] = it->second;
      return QST_OK;
    }
  }
  const std::pair<int, int> pols[] = {{-1, -1}, {1, -1}, {-1, 0}, {1, 0}};
  size_t need = 0;
  for (const auto& p : pols) {
    h->policies[sig] = p;
    size_t nd = 0;
    if (run_call(h, specs, &nd) == QST_OK) need = std::max(need, nd);
  }
  h->last_error.clear();
  st = tune_specs(h, ins, path, al256(need), specs);
  if (st != QST_OK) return st;
  Timer tm;
  double best = -1.0;
  std::pair<int, int> chosen{-1, -1};
  for (const auto& p : pols) {
    h->policies[sig] = p;
    const double ms = time_call(h, specs, tm);
    h->last_error.clear();
    if (ms >= 0 && (best < 0 || ms < best)) {
      best = ms;
      chosen = p;
    }
  }
  if (hipStreamSynchronize(h->stream) != hipSuccess) return set_err(h, QST_ERR_DEVICE, "autotune synchronise failed");
  h->policies[sig] = chosen;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_policy_cache[std::make_pair(h->arch, sig)] = chosen;
  return QST_OK;
}

// A kernel shape exists for the instance: the staged geometry, or else one of the instance-table
// kinds for FP32 Pauli settings with dense frequencies -- fused slices (R 2^n <= 2^14) or the
// on-chip passes (n = 11..14, rows of 16-byte aligned arrays: the instance's, and the call's when
// `call_rows16`).
static qst_status check_shape(qst_handle* h, const qst_instance& in, qst_path path, bool call_rows16 = true) {
  Geometry g;
  const qst_status st = make_geometry(h, in.n_qubits, in.rank, in.n_settings, path, g);
  if (st == QST_OK) return st;
  const bool table = resolve(path) == QST_PATH_BUTTERFLY_F32 && !in.unitaries && !in.freqs_rowptr &&
                     in.settings_per_batch <= 0;
  const bool fits = ((long long)in.rank << in.n_qubits) <= 16384;
  auto a16 = [](const void* p) { return p == nullptr || aligned(p, 16); };
  const bool oc = in.n_qubits >= 11 && in.n_qubits <= 14 && a16(in.atoms) && a16(in.freqs) && a16(in.probs_base) &&
                  call_rows16;
  if (table && (fits || oc)) {
    h->last_error.clear();
    return QST_OK;
  }
  return st;
}

qst_status qst_plan(qst_handle* h, const qst_instance* inst, int n_inst, qst_path path, int autotune) {
  qst_status st = common_checks(h, inst, n_inst, path);
  if (st != QST_OK) return st;
  path = resolve(path);
  for (int i = 0; i < n_inst; ++i) {
    st = validate_instance(h, inst[i], path, false);
    if (st != QST_OK) return st;
    st = check_shape(h, inst[i], path);
    if (st != QST_OK) return st;
  }
  st = device_gate(h);
  if (st != QST_OK) return st;
  if (autotune && !pass_path(path)) {
    if (capturing(h->stream)) return set_err(h, QST_ERR_CAPTURE, "autotune outside stream capture");
    st = n_inst == 1 ? tune_shape(h, inst[0], path) : tune_policy(h, inst, n_inst, path);
    if (st != QST_OK) return st;
  }
  // the same call with these instances, as the compute calls will run it
  size_t need = 0;
  std::vector<RunSpec> specs(n_inst);
  for (int i = 0; i < n_inst; ++i) {
    specs[i].in = &inst[i];
    specs[i].path = path;
    specs[i].adjoint = true;
  }
  st = run_call(h, specs, &need);
  if (st != QST_OK) return st;
  return ensure_ws(h, need);
}

qst_status qst_plan_choice(qst_handle* h, const qst_instance* inst, qst_path path, int set, qst_choice* choice) {
  qst_status st = common_checks(h, inst, 1, path);
  if (st != QST_OK) return st;
  if (!choice) return set_err(h, QST_ERR_INVALID_ARG, "null choice");
  path = resolve(path);
  st = validate_instance(h, *inst, path, false);
  if (st != QST_OK) return st;
  const auto key = shape_key(inst->n_qubits, inst->rank, inst->n_settings, path);
  if (set) {
    if (choice->kind < -1 || choice->kind > 2 || choice->settings_per_batch < 0 || choice->tile_bits_fwd < 0 ||
        choice->tile_bits_adj < 0 || choice->values_per_thread_log2 < 0 || choice->w_row_bits < 0 ||
        choice->w_row_bits > 14 || choice->x_row_bits < 0 || choice->x_row_bits > 14)
      return set_err(h, QST_ERR_INVALID_ARG, "choice fields out of range");
    h->choices[key] = *choice;
    return QST_OK;
  }
  auto it = h->choices.find(key);
  if (it != h->choices.end()) {
    *choice = it->second;
  } else {
    *choice = qst_choice{};
    choice->kind = -1;
  }
  return QST_OK;
}

qst_status qst_forward(qst_handle* h, const qst_instance* inst, int n_inst, void* const* probs, double* loss,
                       qst_loss loss_kind, double eps, qst_path path) {
  qst_status st = common_checks(h, inst, n_inst, path);
  if (st != QST_OK) return st;
  path = resolve(path);
  if (loss_kind < QST_LOSS_CE || loss_kind > QST_LOSS_NONE) return set_err(h, QST_ERR_INVALID_ARG, "bad loss kind");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return set_err(h, QST_ERR_INVALID_ARG, "eps must be finite and >= 0");
  if (loss && loss_kind == QST_LOSS_NONE) return set_err(h, QST_ERR_INVALID_ARG, "loss requested with QST_LOSS_NONE");
  for (int i = 0; i < n_inst; ++i) {
    st = validate_instance(h, inst[i], path, loss != nullptr);
    if (st != QST_OK) return st;
    st = check_shape(h, inst[i], path, !probs || aligned(probs[i], 16));
    if (st != QST_OK) return st;
  }
  st = device_gate(h);
  if (st != QST_OK) return st;
  std::vector<RunSpec> specs(n_inst);
  for (int i = 0; i < n_inst; ++i) {
    RunSpec& rs = specs[i];
    rs.in = &inst[i];
    rs.path = path;
    rs.loss_kind = loss ? loss_kind : QST_LOSS_NONE;
    rs.eps = eps;
    rs.probs = probs ? probs[i] : nullptr;
    rs.loss = loss ? loss + i : nullptr;
    rs.adjoint = false;
  }
  st = run_call(h, specs);
  if (st != QST_OK) return st;
  post_flag(h);
  return QST_OK;
}

static qst_status backward_impl(qst_handle* h, const qst_instance* inst, int n_inst, const void* const* grad_p,
                                void* const* atom_grad, double* const* weight_grad, double* loss, qst_loss loss_kind,
                                double eps, int project_tangent, qst_path path) {
  qst_status st = common_checks(h, inst, n_inst, path);
  if (st != QST_OK) return st;
  path = resolve(path);
  if (loss_kind < QST_LOSS_CE || loss_kind > QST_LOSS_NONE) return set_err(h, QST_ERR_INVALID_ARG, "bad loss kind");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return set_err(h, QST_ERR_INVALID_ARG, "eps must be finite and >= 0");
  if (!atom_grad) return set_err(h, QST_ERR_INVALID_ARG, "atom_grad required");
  if (grad_p && loss_kind != QST_LOSS_NONE)
    return set_err(h, QST_ERR_INVALID_ARG, "grad_p given: loss_kind must be QST_LOSS_NONE");
  if (!grad_p && loss_kind == QST_LOSS_NONE) return set_err(h, QST_ERR_INVALID_ARG, "no loss and no grad_p");
  if (grad_p && loss) return set_err(h, QST_ERR_INVALID_ARG, "loss requested with grad_p");
  for (int i = 0; i < n_inst; ++i) {
    st = validate_instance(h, inst[i], path, grad_p == nullptr);
    if (st != QST_OK) return st;
    if (!atom_grad[i]) return set_err(h, QST_ERR_INVALID_ARG, "null atom_grad entry");
    if (grad_p && !grad_p[i]) return set_err(h, QST_ERR_INVALID_ARG, "null grad_p entry");
    const size_t ea = path == QST_PATH_BUTTERFLY_F64 ? 16 : 8;
    if (!aligned(atom_grad[i], ea)) return set_err(h, QST_ERR_ALIGN, "atom_grad misaligned");
    if (atom_grad[i] == inst[i].atoms) return set_err(h, QST_ERR_INVALID_ARG, "atom_grad aliases atoms");
    st = check_shape(h, inst[i], path, aligned(atom_grad[i], 16) && (!grad_p || aligned(grad_p[i], 16)));
    if (st != QST_OK) return st;
  }
  st = device_gate(h);
  if (st != QST_OK) return st;
  std::vector<RunSpec> specs(n_inst);
  for (int i = 0; i < n_inst; ++i) {
    RunSpec& rs = specs[i];
    rs.in = &inst[i];
    rs.path = path;
    rs.loss_kind = loss_kind;
    rs.eps = eps;
    rs.grad_p = grad_p ? grad_p[i] : nullptr;
    rs.atom_grad = atom_grad[i];
    rs.weight_grad = weight_grad ? weight_grad[i] : nullptr;
    rs.loss = loss ? loss + i : nullptr;
    rs.project_tangent = project_tangent;
    rs.adjoint = true;
  }
  if (h->static_ws) {
    // everything must fit the static scratch before anything is enqueued
    size_t need = 0;
    st = run_call(h, specs, &need);
    if (st != QST_OK) return st;
    st = ensure_ws(h, need);
    if (st != QST_OK) return st;
  }
  st = run_call(h, specs);
  if (st != QST_OK) return st;
  post_flag(h);
  return QST_OK;
}

qst_status qst_backward(qst_handle* h, const qst_instance* inst, int n_inst, const void* const* grad_p,
                        void* const* atom_grad, double* const* weight_grad, double* loss, qst_loss loss_kind,
                        double eps, int project_tangent, qst_path path) {
  return backward_impl(h, inst, n_inst, grad_p, atom_grad, weight_grad, loss, loss_kind, eps, project_tangent, path);
}

qst_status qst_backward_static(qst_handle* h, const qst_instance* inst, int n_inst, const void* const* grad_p,
                               void* const* atom_grad, double* const* weight_grad, double* loss, qst_loss loss_kind,
                               double eps, int project_tangent, qst_path path) {
  if (!h) return QST_ERR_INVALID_ARG;
  if (h->device >= 0 && h->static_scratch == nullptr)
    return set_err(h, QST_ERR_DEVICE, "the static scratch of this device has no address (hipGetSymbolAddress failed)");
  // The handle's own workspace is set aside for the call and the device's static scratch
  // takes its place; ensure_ws then refuses to grow instead of allocating.
  void* const ws = h->ws;
  const size_t ws_bytes = h->ws_bytes;
  h->ws = h->static_scratch;
  h->ws_bytes = h->device >= 0 ? kStaticScratchBytes : 0;
  h->static_ws = true;
  const qst_status st =
      backward_impl(h, inst, n_inst, grad_p, atom_grad, weight_grad, loss, loss_kind, eps, project_tangent, path);
  h->static_ws = false;
  h->ws = ws;
  h->ws_bytes = ws_bytes;
  return st;
}

qst_status qst_atom_trial(qst_handle* h, const qst_instance* inst, int r, const void* psi_trial,
                          const void* probs_t, void* probs_trial, double* loss_trial, qst_loss loss_kind,
                          double eps, qst_path path) {
  qst_status st = common_checks(h, inst, 1, path);
  if (st != QST_OK) return st;
  path = resolve(path);
  if (loss_kind < QST_LOSS_CE || loss_kind > QST_LOSS_NONE) return set_err(h, QST_ERR_INVALID_ARG, "bad loss kind");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return set_err(h, QST_ERR_INVALID_ARG, "eps must be finite and >= 0");
  if (loss_trial && loss_kind == QST_LOSS_NONE)
    return set_err(h, QST_ERR_INVALID_ARG, "loss requested with QST_LOSS_NONE");
  st = validate_instance(h, *inst, path, loss_trial != nullptr);
  if (st != QST_OK) return st;
  if (inst->probs_base) return set_err(h, QST_ERR_INVALID_ARG, "probs_base must be NULL (probs_t is the base)");
  if (r < 0 || r >= inst->rank) return set_err(h, QST_ERR_INVALID_ARG, "atom index out of range");
  if (!psi_trial) return set_err(h, QST_ERR_INVALID_ARG, "null psi_trial");
  const int elem = elem_of(path);
  if (!aligned(psi_trial, 2 * (size_t)elem) || (probs_t && !aligned(probs_t, elem)) ||
      (probs_trial && !aligned(probs_trial, elem)))
    return set_err(h, QST_ERR_ALIGN, "psi_trial/probs_t/probs_trial not aligned to their element size");
  if (probs_trial && (probs_trial == probs_t || probs_trial == inst->atoms))
    return set_err(h, QST_ERR_INVALID_ARG, "probs_trial aliases probs_t or the atoms");
  Geometry g;
  st = make_geometry(h, inst->n_qubits, 2, inst->n_settings, path, g);
  if (st != QST_OK) return st;
  mark(g, *inst);
  st = device_gate(h);
  if (st != QST_OK) return st;

  // The pair (psi_trial, psi_r) and its weights sit at the start of the workspace;
  // the two-atom pass lays out its own buffers after them.  The workspace is sized
  // for both before anything is enqueued, so no reallocation can drop the pair.
  const size_t pair_bytes = al256((size_t)2 * g.D * 2 * elem);
  const size_t base = al256(pair_bytes + 2 * sizeof(double));
  qst_instance pair = *inst;
  pair.rank = 2;
  pair.probs_base = probs_t;
  {
    Geometry gp = g;
    const int S = batch_size(h, gp, pair, path, 0);
    set_grid(h, gp, S);
    st = ensure_ws(h, layout_ws(gp, S, path, false, base).total);
    if (st != QST_OK) return st;
  }
  unsigned char* ws = reinterpret_cast<unsigned char*>(h->ws);
  double* wpair = reinterpret_cast<double*>(ws + pair_bytes);
  pair.atoms = ws;
  pair.weights = wpair;
  prof_begin(h, PK_OTHER);
  QST_HIP(qst::launch_atom_pair(elem, psi_trial, inst->atoms, inst->weights, r, g.D, ws, wpair, h->stream));
  prof_end(h);
  RunSpec rs{};
  rs.in = &pair;
  rs.path = path;
  rs.loss_kind = loss_trial ? loss_kind : QST_LOSS_NONE;
  rs.eps = eps;
  rs.probs = probs_trial;
  rs.loss = loss_trial;
  rs.adjoint = false;
  st = run_instance(h, rs, base);
  if (st != QST_OK) return st;
  post_flag(h);
  return QST_OK;
}

qst_status qst_reweight_simplex(qst_handle* h, const double* alpha, const double* hvec, int R, double eta_alpha,
                                double tau, double* alpha_out, int32_t* keep_idx, int32_t* R_out) {
  if (!h) return QST_ERR_INVALID_ARG;
  h->last_error.clear();
  if (!alpha || !hvec || !alpha_out || !keep_idx || !R_out) return set_err(h, QST_ERR_INVALID_ARG, "null pointer");
  if (R < 1 || R > 1024) return set_err(h, QST_ERR_SHAPE, "R must be in 1..1024");
  if (!std::isfinite(eta_alpha) || !std::isfinite(tau)) return set_err(h, QST_ERR_INVALID_ARG, "non-finite eta/tau");
  if (!aligned(alpha, 8) || !aligned(hvec, 8) || !aligned(alpha_out, 8) || !aligned(keep_idx, 4) || !aligned(R_out, 4))
    return set_err(h, QST_ERR_ALIGN, "misaligned pointer");
  if (h->device < 0) return set_err(h, QST_ERR_UNSUPPORTED, "validation-only handle (device -1): arguments are valid");
  if (hipSetDevice(h->device) != hipSuccess) return set_err(h, QST_ERR_DEVICE, "hipSetDevice failed");
  QST_HIP(qst::launch_reweight(alpha, hvec, R, eta_alpha, tau, alpha_out, keep_idx, R_out, h->stream));
  return QST_OK;
}

qst_status qst_refactor(qst_handle* h, const qst_instance* inst, qst_loss loss_kind, double eps, double eta_rho,
                        double mu, double tau, int L_max, int n_lanczos, const void* v0, void* atoms_out,
                        double* weights_out, int32_t* R_out, int32_t* s_star, double* ritz_vals, double* ritz_resid,
                        double* q_scores, qst_path path) {
  qst_status st = common_checks(h, inst, 1, path);
  if (st != QST_OK) return st;
  path = resolve(path);
  if (path != QST_PATH_BUTTERFLY_F32 && path != QST_PATH_BUTTERFLY_F64)
    return set_err(h, QST_ERR_UNSUPPORTED, "refactor runs on the butterfly paths");
  if (loss_kind != QST_LOSS_CE && loss_kind != QST_LOSS_LS)
    return set_err(h, QST_ERR_INVALID_ARG, "refactor needs a loss (CE or LS)");
  if (!v0 || !atoms_out || !weights_out || !R_out || !s_star || !ritz_vals || !ritz_resid || !q_scores)
    return set_err(h, QST_ERR_INVALID_ARG, "null output pointer");
  if (L_max < 1 || L_max > 64 || n_lanczos < 1 || n_lanczos > 256)
    return set_err(h, QST_ERR_SHAPE, "L_max must be in 1..64 and n_lanczos in 1..256");
  if (!(eta_rho > 0.0) || !std::isfinite(eta_rho) || !std::isfinite(mu) || !std::isfinite(tau) || !(eps >= 0.0))
    return set_err(h, QST_ERR_INVALID_ARG, "bad eta_rho/mu/tau/eps");
  st = validate_instance(h, *inst, path, true);
  if (st != QST_OK) return st;
  {
    Geometry gchk;
    st = make_geometry(h, inst->n_qubits, inst->rank, inst->n_settings, path, gchk);
    if (st != QST_OK) return st;
  }
  st = device_gate(h);
  if (st != QST_OK) return st;
  const int elem = elem_of(path);
  const bool c64 = elem == 4;
  const int n = inst->n_qubits, R = inst->rank, B = inst->n_settings;
  const long long D = 1ll << n;
  Geometry gR, g1;
  st = make_geometry(h, n, R, B, path, gR);
  if (st != QST_OK) return st;
  st = make_geometry(h, n, 1, B, path, g1);
  if (st != QST_OK) return st;
  mark(gR, *inst);
  mark(g1, *inst);
  const int k_max = (int)std::min<long long>(n_lanczos, D);
  hipStream_t s = h->stream;

  // Workspace: [run region for R atoms | run region for one vector | gneg | Krylov Q | w | vin | gv | A128 | misc]
  const int SR = default_S(gR);
  set_grid(h, gR, SR);
  const WsLayout LR = layout_ws(gR, SR, path, true, 0);
  const int S1 = default_S(g1);
  set_grid(h, g1, S1);
  const WsLayout L1 = layout_ws(g1, S1, path, false, al256(LR.total));
  size_t o = al256(L1.total);
  const size_t off_Q = o;
  o = al256(o + (size_t)(k_max + 1) * D * 16);
  const size_t off_w = o;
  o = al256(o + (size_t)D * 16);
  const size_t off_vin = o;
  o = al256(o + (size_t)D * 2 * elem);
  const size_t off_gv = o;
  o = al256(o + (size_t)D * 2 * elem);
  const size_t off_A = o;
  o = al256(o + (size_t)R * D * 16);
  const size_t off_misc = o;
  o = al256(o + 64 * 1024);
  const size_t off_dpart = o;
  o = al256(o + (size_t)(k_max + R + 2) * G1 * 2 * 8);
  // G v with the settings grouped by their high codes (one vector, FP32, Pauli settings,
  // 14 low bits): pattern code words, member code words, member order, group starts and the
  // patterns' settings rows.
  const bool grouped = gv_grouped_on() && c64 && !inst->unitaries && g1.n_hi > 0 && g1.n_mid == 0 && g1.n_lo == qst::kGvLoBits;
  const size_t off_grp = o;
  if (grouped) o = al256(o + (size_t)B * 8 * 2 + (size_t)B * 4 * 2 + 4 + (size_t)B * n + 256);
  st = ensure_ws(h, o);
  if (st != QST_OK) return st;
  unsigned char* ws = reinterpret_cast<unsigned char*>(h->ws);
  void* gneg = ws + LR.gneg;
  double2* Q = reinterpret_cast<double2*>(ws + off_Q);
  double2* w = reinterpret_cast<double2*>(ws + off_w);
  void* vin = ws + off_vin;
  void* gv = ws + off_gv;
  double2* A128 = reinterpret_cast<double2*>(ws + off_A);
  double* misc = reinterpret_cast<double*>(ws + off_misc);  // [0..1]: alpha=1; [16..]: coef/dots
  double* dpart = reinterpret_cast<double*>(ws + off_dpart);
  double* dots = misc + 16;
  double* coef = misc + 16 + 2 * 512;
  h->prof_outer = false;

  // 1. -g of the current state (dL/dp), written by the forward pass.
  {
    RunSpec rs{};
    rs.in = inst;
    rs.path = path;
    rs.loss_kind = loss_kind;
    rs.eps = eps;
    rs.gneg = gneg;
    rs.adjoint = false;
    rs.S_override = SR;
    st = run_instance(h, rs, 0, nullptr);
    if (st != QST_OK) return st;
  }
  // Grouping of the settings by their high codes (qubits 0 .. n_hi - 1, i.e. index bits
  // n - 1 .. n_lo; codes above 2 read as Z, as the decode does).
  int n_pat = 0;
  uint64_t *pc_pat = nullptr, *pc_all = nullptr;
  int *perm_d = nullptr, *goff_d = nullptr;
  if (grouped) {
    unsigned char* gb = ws + off_grp;
    pc_pat = reinterpret_cast<uint64_t*>(gb);
    pc_all = pc_pat + B;
    perm_d = reinterpret_cast<int*>(pc_all + B);
    goff_d = perm_d + B;
    uint8_t* set_pat = reinterpret_cast<uint8_t*>(goff_d + B + 1);
    std::vector<uint8_t> sh((size_t)B * n);
    QST_HIP(hipMemcpyAsync(sh.data(), inst->settings, sh.size(), hipMemcpyDeviceToHost, s));
    QST_HIP(hipStreamSynchronize(s));
    const int nh = g1.n_hi;
    std::vector<uint32_t> key(B);
    for (int bb = 0; bb < B; ++bb) {
      uint32_t kk = 0;
      for (int j = 0; j < nh; ++j) kk = kk * 3u + std::min<uint32_t>(sh[(size_t)bb * n + j], 2u);
      key[bb] = kk;
    }
    std::vector<int> perm(B), goff;
    for (int bb = 0; bb < B; ++bb) perm[bb] = bb;
    std::stable_sort(perm.begin(), perm.end(), [&](int x, int y) { return key[x] < key[y]; });
    std::vector<uint8_t> sp;
    for (int i = 0; i < B; ++i) {
      if (i > 0 && key[perm[i]] == key[perm[i - 1]]) continue;
      goff.push_back(i);
      for (int j = 0; j < n; ++j) sp.push_back(j < nh ? std::min<uint8_t>(sh[(size_t)perm[i] * n + j], 2) : 2);
    }
    n_pat = (int)goff.size();
    goff.push_back(B);
    QST_HIP(hipMemcpyAsync(perm_d, perm.data(), (size_t)B * 4, hipMemcpyHostToDevice, s));
    QST_HIP(hipMemcpyAsync(goff_d, goff.data(), goff.size() * 4, hipMemcpyHostToDevice, s));
    QST_HIP(hipMemcpyAsync(set_pat, sp.data(), sp.size(), hipMemcpyHostToDevice, s));
    QST_HIP(qst::launch_decode(set_pat, n_pat, n, pc_pat, h->dflag, s));
    QST_HIP(qst::launch_decode(inst->settings, B, n, pc_all, h->dflag, s));
    QST_HIP(hipStreamSynchronize(s));  // the host vectors above go out of scope
  }
  // One G v product, gv = sum_b V_b^dagger diag(2^-k_b (-g_b)) V_b vin: grouped (stage A on
  // the patterns, the grouped low stage, stage C on the patterns) or through the staged path.
  auto gv_product = [&]() -> qst_status {
    if (!grouped) {
      qst_instance one_inst = *inst;
      one_inst.rank = 1;
      one_inst.atoms = vin;
      one_inst.weights = misc;
      RunSpec rs{};
      rs.in = &one_inst;
      rs.path = path;
      rs.loss_kind = QST_LOSS_NONE;
      rs.grad_p = gneg;
      rs.atom_grad = gv;
      rs.adjoint = true;
      rs.S_override = S1;
      return run_instance(h, rs, L1.pc, nullptr);
    }
    void* XP = ws + L1.X;
    void* WP = ws + L1.W;
    const int gv_grid_max = h->num_cu * gv_occ(h);
    for (int p0 = 0; p0 < n_pat; p0 += S1) {
      const int Sp = std::min(S1, n_pat - p0);
      qst::HiArgs ha{};
      ha.src = vin;
      ha.dst = XP;
      ha.pc = pc_pat;
      ha.D = D;
      ha.R = 1;
      ha.n = n;
      ha.n_lo = g1.n_lo;
      ha.n_hi = g1.n_hi;
      ha.t = g1.t;
      ha.c = g1.c;
      ha.b0 = p0;
      ha.S = Sp;
      ha.nsplit = split_of(h, g1, g1.c, Sp);
      QST_HIP(qst::launch_stage_hi(g1, ha, false, s));
      qst::GvArgs ga{};
      ga.X = reinterpret_cast<const float2*>(XP);
      ga.W = reinterpret_cast<float2*>(WP);
      ga.pc = pc_all;
      ga.perm = perm_d;
      ga.goff = goff_d;
      ga.g = reinterpret_cast<const float*>(gneg);
      ga.alpha = misc;
      ga.n = n;
      ga.p0 = p0;
      ga.S = Sp;
      const int grid = (int)std::min<long long>((long long)Sp << g1.n_hi, gv_grid_max);
      QST_HIP(qst::launch_gv_lo(ga, 5, grid, s));
      qst::HiArgs hc{};
      hc.src = WP;
      hc.dst = gv;
      hc.pc = pc_pat;
      hc.D = D;
      hc.R = 1;
      hc.n = n;
      hc.n_lo = g1.n_lo;
      hc.n_hi = g1.n_hi;
      hc.t = g1.t_adj;
      hc.c = g1.c_adj;
      hc.b0 = p0;
      hc.S = Sp;
      hc.first = p0 == 0;
      hc.nsplit = std::min(g1.split_adj, split_of(h, g1, g1.c_adj, Sp));
      hc.part = ws + L1.split;
      Geometry gc = g1;
      gc.t = g1.t_adj;
      gc.c = g1.c_adj;
      QST_HIP(qst::launch_stage_hi(gc, hc, true, s));
      if (hc.nsplit > 1) QST_HIP(qst::launch_sum_splits(4, hc.part, hc.nsplit, D, gv, hc.first, s));
    }
    return QST_OK;
  };

  // Atoms in complex128 for the low-rank term, and the unit weight of the G v products.
  QST_HIP(qst::launch_convert(inst->atoms, c64, A128, 0, (long long)R * D, 1.0, s));
  std::vector<double> alpha_h(R);
  QST_HIP(hipMemcpyAsync(alpha_h.data(), inst->weights, R * sizeof(double), hipMemcpyDeviceToHost, s));
  const double one = 1.0;
  QST_HIP(hipMemcpyAsync(misc, &one, sizeof(double), hipMemcpyHostToDevice, s));

  auto dots_host = [&](const double2* rows, int k, const void* x, int x_c64, std::vector<double>& out) -> qst_status {
    QST_HIP(qst::launch_dots(rows, k, D, x, x_c64, D, dpart, G1, dots, s));
    out.resize(2 * k);
    QST_HIP(hipMemcpyAsync(out.data(), dots, 2 * k * sizeof(double), hipMemcpyDeviceToHost, s));
    QST_HIP(hipStreamSynchronize(s));
    return QST_OK;
  };

  // q_0 = v0 / ||v0||
  QST_HIP(qst::launch_convert(v0, 0, Q, 0, D, 1.0, s));
  std::vector<double> tmp;
  st = dots_host(Q, 1, Q, 0, tmp);
  if (st != QST_OK) return st;
  const double nv0 = std::sqrt(tmp[0]);
  if (!(nv0 > 0.0) || !std::isfinite(nv0)) return set_err(h, QST_ERR_INVALID_ARG, "v0 must be non-zero and finite");
  QST_HIP(qst::launch_convert(Q, 0, Q, 0, D, 1.0 / nv0, s));

  std::vector<double> a, b;
  double scale = 0.0;
  int k = 0;
  for (int j = 0; j < k_max; ++j) {
    double2* qj = Q + (size_t)j * D;
    // low-rank term: sum_r alpha_r psi_r <psi_r, q_j>
    st = dots_host(A128, R, qj, 0, tmp);
    if (st != QST_OK) return st;
    std::vector<double> cf(2 * R);
    for (int r = 0; r < R; ++r) {
      cf[2 * r] = alpha_h[r] * tmp[2 * r];
      cf[2 * r + 1] = alpha_h[r] * tmp[2 * r + 1];
    }
    QST_HIP(hipMemcpyAsync(coef, cf.data(), cf.size() * sizeof(double), hipMemcpyHostToDevice, s));
    QST_HIP(qst::launch_fill(w, (size_t)D * 16, s));
    QST_HIP(qst::launch_combine(w, A128, R, D, coef, 1.0, 0, D, s));
    // eta_rho G q_j: adjoint pass with one unit-weight atom and sensitivity -g
    QST_HIP(qst::launch_convert(qj, 0, vin, c64, D, 1.0, s));
    prof_outer_begin(h);
    st = gv_product();
    prof_outer_end(h);
    if (st != QST_OK) return st;
    QST_HIP(qst::launch_axpy_c(w, 0, gv, c64, D, eta_rho, s));
    // a_j = Re <q_j, w>
    st = dots_host(qj, 1, w, 0, tmp);
    if (st != QST_OK) return st;
    const double aj = tmp[0];
    // w -= b_{j-1} q_{j-1} + a_j q_j   (rows q_{j-1}, q_j are adjacent in Q)
    if (j > 0) {
      cf.assign({b[j - 1], 0.0, aj, 0.0});
      QST_HIP(hipMemcpyAsync(coef, cf.data(), 4 * sizeof(double), hipMemcpyHostToDevice, s));
      QST_HIP(qst::launch_combine(w, Q + (size_t)(j - 1) * D, 2, D, coef, -1.0, 0, D, s));
    } else {
      cf.assign({aj, 0.0});
      QST_HIP(hipMemcpyAsync(coef, cf.data(), 2 * sizeof(double), hipMemcpyHostToDevice, s));
      QST_HIP(qst::launch_combine(w, qj, 1, D, coef, -1.0, 0, D, s));
    }
    // full re-orthogonalisation, twice
    for (int pass = 0; pass < 2; ++pass) {
      QST_HIP(qst::launch_dots(Q, j + 1, D, w, 0, D, dpart, G1, dots, s));
      QST_HIP(qst::launch_combine(w, Q, j + 1, D, dots, -1.0, 0, D, s));
    }
    st = dots_host(w, 1, w, 0, tmp);
    if (st != QST_OK) return st;
    const double bj = std::sqrt(std::max(tmp[0], 0.0));
    a.push_back(aj);
    b.push_back(bj);
    k = j + 1;
    scale = std::max(scale, std::max(std::fabs(aj), bj));
    if (j + 1 == k_max || bj <= 1e-13 * std::max(scale, 1e-300)) break;
    QST_HIP(qst::launch_convert(w, 0, Q + (size_t)(j + 1) * D, 0, D, 1.0 / bj, s));
  }

  // Tridiagonal eigenproblem on the host (FP64).
  std::vector<double> T((size_t)k * k, 0.0), ev, Y;
  for (int i = 0; i < k; ++i) {
    T[(size_t)i * k + i] = a[i];
    if (i + 1 < k) T[(size_t)i * k + i + 1] = T[(size_t)(i + 1) * k + i] = b[i];
  }
  jacobi_eigh(T, k, ev, Y);
  std::vector<int> order(k);
  for (int i = 0; i < k; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return ev[x] > ev[y]; });
  const int L = std::min(L_max, k);
  std::vector<double> theta(L), resid(L);
  for (int l = 0; l < L; ++l) {
    theta[l] = ev[order[l]];
    resid[l] = std::fabs(b[k - 1] * Y[(size_t)(k - 1) * k + order[l]]);
  }
  // Candidates s = 1..L: beta = proj(theta_1..s), prune, score.
  std::vector<double> scores(L);
  std::vector<std::vector<int>> keeps(L);
  std::vector<std::vector<double>> wts(L);
  for (int sidx = 0; sidx < L; ++sidx) {
    std::vector<double> lam(theta.begin(), theta.begin() + sidx + 1);
    std::vector<double> beta = proj_simplex(lam);
    std::vector<int> keep;
    double sum = 0.0;
    for (int i = 0; i <= sidx; ++i)
      if (beta[i] > tau) {
        keep.push_back(i);
        sum += beta[i];
      }
    if (keep.empty()) {
      int arg = 0;
      for (int i = 1; i <= sidx; ++i)
        if (beta[i] > beta[arg]) arg = i;
      keep.push_back(arg);
      sum = beta[arg];
    }
    std::vector<double> bc;
    double sq = 0.0, lin = 0.0;
    for (int i : keep) {
      bc.push_back(beta[i] / sum);
      sq += (beta[i] / sum) * (beta[i] / sum);
      lin += (beta[i] / sum) * theta[i];
    }
    scores[sidx] = (sq - 2.0 * lin) / (2.0 * eta_rho) + mu * (double)keep.size();
    keeps[sidx] = keep;
    wts[sidx] = bc;
  }
  int best = 0;
  for (int i = 1; i < L; ++i)
    if (scores[i] < scores[best]) best = i;
  const std::vector<int>& keep = keeps[best];
  const int Rout = (int)keep.size();

  // Ritz vectors of the chosen candidate: phi_l = sum_j Y[j][l] q_j, written to atoms_out.
  QST_HIP(qst::launch_fill(atoms_out, (size_t)L_max * D * 2 * elem, s));
  for (int i = 0; i < Rout; ++i) {
    std::vector<double> cf(2 * k, 0.0);
    for (int j = 0; j < k; ++j) cf[2 * j] = Y[(size_t)j * k + order[keep[i]]];
    QST_HIP(hipMemcpyAsync(coef, cf.data(), cf.size() * sizeof(double), hipMemcpyHostToDevice, s));
    QST_HIP(qst::launch_fill(w, (size_t)D * 16, s));
    QST_HIP(qst::launch_combine(w, Q, k, D, coef, 1.0, 0, D, s));
    QST_HIP(qst::launch_convert(w, 0, reinterpret_cast<unsigned char*>(atoms_out) + (size_t)i * D * 2 * elem, c64, D,
                                1.0, s));
    QST_HIP(hipStreamSynchronize(s));  // coef is reused by the next row
  }
  std::vector<double> wout(L_max, 0.0), rv(L_max, 0.0), rr(L_max, 0.0), qs(L_max, 0.0);
  for (int i = 0; i < Rout; ++i) wout[i] = wts[best][i];
  for (int l = 0; l < L; ++l) {
    rv[l] = theta[l];
    rr[l] = resid[l];
    qs[l] = scores[l];
  }
  const int32_t ro = Rout, sb = best;
  QST_HIP(hipMemcpyAsync(weights_out, wout.data(), L_max * sizeof(double), hipMemcpyHostToDevice, s));
  QST_HIP(hipMemcpyAsync(ritz_vals, rv.data(), L_max * sizeof(double), hipMemcpyHostToDevice, s));
  QST_HIP(hipMemcpyAsync(ritz_resid, rr.data(), L_max * sizeof(double), hipMemcpyHostToDevice, s));
  QST_HIP(hipMemcpyAsync(q_scores, qs.data(), L_max * sizeof(double), hipMemcpyHostToDevice, s));
  QST_HIP(hipMemcpyAsync(R_out, &ro, sizeof(int32_t), hipMemcpyHostToDevice, s));
  QST_HIP(hipMemcpyAsync(s_star, &sb, sizeof(int32_t), hipMemcpyHostToDevice, s));
  QST_HIP(hipStreamSynchronize(s));
  post_flag(h);
  return QST_OK;
}

}  // extern "C"
