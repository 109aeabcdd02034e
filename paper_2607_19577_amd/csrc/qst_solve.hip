// Host driver of the rank-adaptive iteration (Algorithm 1) and the Gram-form state
// error.  Every oracle call runs on the device through the public entry points
// (forward, fused backward, atom-step response, coefficient step, spectral
// refactorisation); the host keeps the slot schedule, the step-size search and the
// acceptance tests, which need one scalar per trial.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <utility>
#include <vector>

#include "qst.h"
#include "qst_host.hpp"
#include "qst_internal.hpp"

namespace {

// Device memory released when the driver returns (also on an error path).
struct DevBuf {
  void* p = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() {
    if (p) (void)hipFree(p);  // release on every path; a failure here has nothing to report to
  }
  hipError_t alloc(size_t bytes) { return hipMalloc(&p, bytes ? bytes : 1); }
  template <typename T>
  T* as() const {
    return reinterpret_cast<T*>(p);
  }
};

enum { KIND_RHO = 0, KIND_ALPHA = 1, KIND_PSI = 2 };

int slot_kind(int t, int t_alpha, int t_ref) {
  if (t_ref > 0 && t % t_ref == 0) return KIND_RHO;
  if (t_alpha > 0 && t % t_alpha == 0) return KIND_ALPHA;
  return KIND_PSI;
}

bool finite_nonneg(double x) { return std::isfinite(x) && x >= 0.0; }

}  // namespace

#define QST_S_HIP(expr)                                                                         \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess)                                                                       \
      return qst_host_error(h, QST_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define QST_S_CALL(expr)       \
  do {                         \
    qst_status s_ = (expr);    \
    if (s_ != QST_OK) return s_; \
  } while (0)

extern "C" qst_status qst_solve(qst_handle* h, const qst_instance* inst, const qst_solve_params* prm,
                                const void* v0s, int n_v0, void* atoms_out, double* weights_out, int32_t* rank_out,
                                double* history, int64_t* info, qst_path path) {
  if (!h) return QST_ERR_INVALID_ARG;
  if (!inst || !prm) return qst_host_error(h, QST_ERR_INVALID_ARG, "null instance or parameters");
  const qst_solve_params P = *prm;
  if (P.max_slots < 0 || P.t_alpha < 0 || P.t_ref < 0 || P.stop_window < 0 || P.oracle_budget < 0)
    return qst_host_error(h, QST_ERR_INVALID_ARG, "negative schedule or stopping parameter");
  if (P.n_grid < 1 || P.n_grid > 60) return qst_host_error(h, QST_ERR_INVALID_ARG, "n_grid must be in 1..60");
  if (P.rank_max < 1 || P.rank_max > 16) return qst_host_error(h, QST_ERR_SHAPE, "rank_max must be in 1..16");
  if (P.n_lanczos < 1) return qst_host_error(h, QST_ERR_INVALID_ARG, "n_lanczos must be >= 1");
  if (P.loss_kind != QST_LOSS_CE && P.loss_kind != QST_LOSS_LS)
    return qst_host_error(h, QST_ERR_INVALID_ARG, "loss_kind must be QST_LOSS_CE or QST_LOSS_LS");
  if (!finite_nonneg(P.mu) || !finite_nonneg(P.eps) || !finite_nonneg(P.tau) || !finite_nonneg(P.tau_acc) ||
      !std::isfinite(P.stop_delta))
    return qst_host_error(h, QST_ERR_INVALID_ARG, "mu, eps, tau, tau_acc must be finite and >= 0");
  if (inst->rank < 1 || inst->rank > P.rank_max)
    return qst_host_error(h, QST_ERR_SHAPE, "initial rank must be in 1..rank_max");
  if (!inst->freqs) return qst_host_error(h, QST_ERR_INVALID_ARG, "freqs required");
  if (inst->probs_base) return qst_host_error(h, QST_ERR_INVALID_ARG, "probs_base must be NULL");
  if (P.t_ref > 0 && (!v0s || n_v0 < 1))
    return qst_host_error(h, QST_ERR_INVALID_ARG, "spectral slots need Lanczos start vectors (v0s, n_v0 >= 1)");
  if (!atoms_out || !weights_out || !rank_out) return qst_host_error(h, QST_ERR_INVALID_ARG, "null output");
  if (inst->n_qubits < 1 || inst->n_qubits > 20 || inst->n_settings < 1)
    return qst_host_error(h, QST_ERR_SHAPE, "n_qubits must be in 1..20 and n_settings >= 1");
  if (path == QST_PATH_AUTO) path = QST_PATH_BUTTERFLY_F32;
  if (qst_host_device(h) < 0)
    return qst_host_error(h, QST_ERR_UNSUPPORTED, "validation-only handle (device -1): arguments are valid");

  const qst_loss loss = (qst_loss)P.loss_kind;
  const int elem = path == QST_PATH_BUTTERFLY_F64 ? 8 : 4;
  const size_t cb = 2 * (size_t)elem;  // bytes per complex
  const long long D = 1ll << inst->n_qubits;
  const long long B = inst->n_settings;
  const int cap = P.rank_max;
  const size_t rows_bytes = (size_t)cap * D * cb;
  const size_t probs_bytes = (size_t)B * D * elem;
  hipStream_t st = qst_host_stream(h);

  DevBuf atA, atB, wA, wB, pA, pB, gfull, gpair, pair, pairw, trial, small, ritz;
  QST_S_HIP(atA.alloc(rows_bytes));
  QST_S_HIP(atB.alloc(rows_bytes));
  QST_S_HIP(wA.alloc((size_t)cap * 8));
  QST_S_HIP(wB.alloc((size_t)cap * 8));
  QST_S_HIP(pA.alloc(probs_bytes));
  QST_S_HIP(pB.alloc(probs_bytes));
  QST_S_HIP(gfull.alloc(rows_bytes));
  QST_S_HIP(gpair.alloc(2 * (size_t)D * cb));
  QST_S_HIP(pair.alloc(2 * (size_t)D * cb));
  QST_S_HIP(pairw.alloc(2 * 8));
  QST_S_HIP(trial.alloc((size_t)D * cb));
  // small scalars: loss, sumsq, R_out, s_star, keep[cap], wgrad[cap], part[kTrialBlocks], lvl1[256]
  const size_t o_loss = 0, o_sumsq = 8, o_rout = 16, o_sstar = 24, o_keep = 32;
  const size_t o_wgrad = o_keep + (((size_t)cap * 4 + 7) & ~(size_t)7);
  const size_t o_part = o_wgrad + (size_t)cap * 8;
  const size_t o_lvl1 = o_part + (size_t)qst::kTrialBlocks * 8;
  const size_t small_bytes = o_lvl1 + 256 * 8;
  QST_S_HIP(small.alloc(small_bytes));
  QST_S_HIP(ritz.alloc((size_t)3 * cap * 8));
  unsigned char* sm = small.as<unsigned char>();
  double* d_loss = reinterpret_cast<double*>(sm + o_loss);
  double* d_sumsq = reinterpret_cast<double*>(sm + o_sumsq);
  int32_t* d_rout = reinterpret_cast<int32_t*>(sm + o_rout);
  int32_t* d_sstar = reinterpret_cast<int32_t*>(sm + o_sstar);
  int32_t* d_keep = reinterpret_cast<int32_t*>(sm + o_keep);
  double* d_wgrad = reinterpret_cast<double*>(sm + o_wgrad);
  double* d_part = reinterpret_cast<double*>(sm + o_part);
  double* d_lvl1 = reinterpret_cast<double*>(sm + o_lvl1);
  double* d_ritz = ritz.as<double>();

  // current and candidate state; probabilities of the current state in p_cur
  unsigned char* cur = atA.as<unsigned char>();
  unsigned char* cand = atB.as<unsigned char>();
  double* w_cur = wA.as<double>();
  double* w_cand = wB.as<double>();
  void* p_cur = pA.p;
  void* p_cand = pB.p;
  int R = inst->rank;
  QST_S_HIP(hipMemcpyAsync(cur, inst->atoms, (size_t)R * D * cb, hipMemcpyDeviceToDevice, st));
  QST_S_HIP(hipMemcpyAsync(w_cur, inst->weights, (size_t)R * 8, hipMemcpyDeviceToDevice, st));

  auto state = [&](const void* atoms, const double* w, int rank, const void* base) {
    qst_instance x = *inst;
    x.atoms = atoms;
    x.weights = w;
    x.rank = rank;
    x.probs_base = base;
    return x;
  };
  auto read_scalar = [&](const void* dptr, void* host, size_t bytes) -> qst_status {
    QST_S_HIP(hipMemcpyAsync(host, dptr, bytes, hipMemcpyDeviceToHost, st));
    QST_S_HIP(hipStreamSynchronize(st));
    return QST_OK;
  };
  // J = L + mu R of a state; its probabilities go to probs_out.
  auto objective = [&](const void* atoms, const double* w, int rank, void* probs_out, double& J) -> qst_status {
    const qst_instance x = state(atoms, w, rank, nullptr);
    void* pp[1] = {probs_out};
    QST_S_CALL(qst_forward(h, &x, 1, pp, d_loss, loss, P.eps, path));
    double L = 0.0;
    QST_S_CALL(read_scalar(d_loss, &L, 8));
    J = L + P.mu * rank;
    return QST_OK;
  };

  double J = 0.0;
  QST_S_CALL(objective(cur, w_cur, R, p_cur, J));
  std::vector<double> accepted_J{J};
  int64_t n_oracle = 1;
  int n_spectral = 0;
  int stop = 0;
  int slots = 0;
  const int lanczos_products = (int)std::min<long long>(P.n_lanczos, D);

  for (int t = 0; t < P.max_slots; ++t) {
    const int kind = slot_kind(t, P.t_alpha, P.t_ref);
    bool acc = false;
    int j_acc = -1;
    if (kind == KIND_RHO) {
      const void* v0 = reinterpret_cast<const unsigned char*>(v0s) + (size_t)(n_spectral % n_v0) * D * 16;
      ++n_spectral;
      for (int j = 0; j < P.n_grid && !acc; ++j) {
        const double eta = std::ldexp(1.0, -j);
        const qst_instance x = state(cur, w_cur, R, nullptr);
        QST_S_CALL(qst_refactor(h, &x, loss, P.eps, eta, P.mu, P.tau, cap, P.n_lanczos, v0, cand, w_cand, d_rout,
                                d_sstar, d_ritz, d_ritz + cap, d_ritz + 2 * cap, path));
        int32_t Rn = 0;
        QST_S_CALL(read_scalar(d_rout, &Rn, 4));
        if (Rn < 1 || Rn > cap) return qst_host_error(h, QST_ERR_NUMERIC, "spectral step returned an invalid rank");
        double Jn = 0.0;
        QST_S_CALL(objective(cand, w_cand, Rn, p_cand, Jn));
        n_oracle += lanczos_products + 1;
        if (Jn <= J - P.tau_acc) {
          std::swap(cur, cand);
          std::swap(w_cur, w_cand);
          std::swap(p_cur, p_cand);
          R = Rn;
          J = Jn;
          acc = true;
          j_acc = j;
        }
      }
    } else if (kind == KIND_ALPHA) {
      // A^T c = -dL/dalpha from the fused backward; the step takes eta_alpha = -eta on it
      const qst_instance x = state(cur, w_cur, R, nullptr);
      void* ag[1] = {gfull.p};
      double* wg[1] = {d_wgrad};
      QST_S_CALL(qst_backward(h, &x, 1, nullptr, ag, wg, nullptr, loss, P.eps, 0, path));
      ++n_oracle;
      for (int j = 0; j < P.n_grid && !acc; ++j) {
        const double eta = std::ldexp(1.0, -j);
        QST_S_CALL(qst_reweight_simplex(h, w_cur, d_wgrad, R, -eta, P.tau, w_cand, d_keep, d_rout));
        int32_t Rn = 0;
        QST_S_CALL(read_scalar(d_rout, &Rn, 4));
        if (Rn < 1 || Rn > R) return qst_host_error(h, QST_ERR_NUMERIC, "coefficient step returned an invalid rank");
        QST_S_HIP(qst::launch_gather_rows(elem, cur, d_keep, d_rout, cap, D, cand, st));
        double Jn = 0.0;
        QST_S_CALL(objective(cand, w_cand, Rn, p_cand, Jn));
        ++n_oracle;
        if (Jn <= J - P.tau_acc) {
          std::swap(cur, cand);
          std::swap(w_cur, w_cand);
          std::swap(p_cur, p_cand);
          R = Rn;
          J = Jn;
          acc = true;
          j_acc = j;
        }
      }
    } else {
      // Atom step on r = t mod R.  G psi_r through a two-atom instance (psi_r, psi_r) with
      // weights (alpha_r, -alpha_r) on the base p_cur: its p is p_cur exactly, and the
      // first atom's projected gradient is (I - psi_r psi_r^*) dL/dpsi_r^*.
      const int r = t % R;
      const unsigned char* psi_r = cur + (size_t)r * D * cb;
      QST_S_HIP(qst::launch_atom_pair(elem, psi_r, cur, w_cur, r, D, pair.p, pairw.as<double>(), st));
      const qst_instance xp = state(pair.p, pairw.as<double>(), 2, p_cur);
      void* ag[1] = {gpair.p};
      QST_S_CALL(qst_backward(h, &xp, 1, nullptr, ag, nullptr, nullptr, loss, P.eps, 1, path));
      ++n_oracle;
      for (int j = 0; j < P.n_grid && !acc; ++j) {
        const double eta = std::ldexp(1.0, -j);
        // psi~ = (psi_r + eta d) / ||.||, d = -(projected gradient)
        QST_S_HIP(qst::launch_trial_atom(elem, psi_r, gpair.p, -eta, trial.p, D, d_part, d_lvl1, 256, d_sumsq, st));
        const qst_instance x = state(cur, w_cur, R, nullptr);
        QST_S_CALL(qst_atom_trial(h, &x, r, trial.p, p_cur, p_cand, d_loss, loss, P.eps, path));
        double L = 0.0;
        QST_S_CALL(read_scalar(d_loss, &L, 8));
        const double Jn = L + P.mu * R;
        ++n_oracle;
        if (Jn <= J - P.tau_acc) {
          QST_S_HIP(hipMemcpyAsync(cur + (size_t)r * D * cb, trial.p, (size_t)D * cb, hipMemcpyDeviceToDevice, st));
          std::swap(p_cur, p_cand);
          J = Jn;
          acc = true;
          j_acc = j;
        }
      }
    }
    slots = t + 1;
    if (acc) accepted_J.push_back(J);
    if (history) {
      double* hr = history + (size_t)t * 6;
      hr[0] = t;
      hr[1] = kind;
      hr[2] = J;
      hr[3] = R;
      hr[4] = acc ? 1.0 : 0.0;
      hr[5] = j_acc;
    }
    if (P.oracle_budget > 0 && n_oracle >= P.oracle_budget) {
      stop = 2;
      break;
    }
    if (acc && P.stop_window > 0 && accepted_J.size() > (size_t)P.stop_window) {
      const double j0 = accepted_J[accepted_J.size() - 1 - P.stop_window];
      if ((j0 - J) / std::fabs(j0) < P.stop_delta) {
        stop = 1;
        break;
      }
    }
  }

  QST_S_HIP(hipMemcpyAsync(atoms_out, cur, (size_t)R * D * cb, hipMemcpyDeviceToDevice, st));
  if (R < cap)
    QST_S_HIP(qst::launch_fill(reinterpret_cast<unsigned char*>(atoms_out) + (size_t)R * D * cb,
                               (size_t)(cap - R) * D * cb, st));
  QST_S_HIP(hipMemcpyAsync(weights_out, w_cur, (size_t)R * 8, hipMemcpyDeviceToDevice, st));
  if (R < cap) QST_S_HIP(qst::launch_fill(weights_out + R, (size_t)(cap - R) * 8, st));
  QST_S_HIP(hipStreamSynchronize(st));
  *rank_out = R;
  if (info) {
    info[0] = slots;
    info[1] = n_oracle;
    info[2] = stop;
  }
  return QST_OK;
}

extern "C" qst_status qst_state_error(qst_handle* h, int n_qubits, const void* atoms_a, const double* w_a, int R_a,
                                      const void* atoms_b, const double* w_b, int R_b, double* out, qst_path path) {
  if (!h) return QST_ERR_INVALID_ARG;
  if (!atoms_a || !w_a || !atoms_b || !w_b || !out) return qst_host_error(h, QST_ERR_INVALID_ARG, "null argument");
  if (n_qubits < 1 || n_qubits > 20) return qst_host_error(h, QST_ERR_SHAPE, "n_qubits must be in 1..20");
  if (R_a < 1 || R_a > 1024 || R_b < 1 || R_b > 1024) return qst_host_error(h, QST_ERR_SHAPE, "ranks must be in 1..1024");
  if (path == QST_PATH_AUTO) path = QST_PATH_BUTTERFLY_F32;
  if (path < QST_PATH_AUTO || path > QST_PATH_BUTTERFLY_BF16) return qst_host_error(h, QST_ERR_INVALID_ARG, "bad path");
  if (qst_host_device(h) < 0)
    return qst_host_error(h, QST_ERR_UNSUPPORTED, "validation-only handle (device -1): arguments are valid");
  const int c64 = path == QST_PATH_BUTTERFLY_F64 ? 0 : 1;
  const size_t cb = c64 ? 8 : 16;
  const long long D = 1ll << n_qubits;
  constexpr int g1 = 256;
  hipStream_t st = qst_host_stream(h);
  DevBuf qa, qb, part, dots;
  QST_S_HIP(qa.alloc((size_t)R_a * D * 16));
  QST_S_HIP(qb.alloc((size_t)R_b * D * 16));
  const int kmax = std::max(R_a, R_b);
  QST_S_HIP(part.alloc((size_t)kmax * g1 * 2 * 8));
  QST_S_HIP(dots.alloc((size_t)kmax * 2 * 8));
  QST_S_HIP(qst::launch_convert(atoms_a, c64, qa.p, 0, (long long)R_a * D, 1.0, st));
  QST_S_HIP(qst::launch_convert(atoms_b, c64, qb.p, 0, (long long)R_b * D, 1.0, st));
  std::vector<double> wa(R_a), wb(R_b);
  QST_S_HIP(hipMemcpyAsync(wa.data(), w_a, (size_t)R_a * 8, hipMemcpyDeviceToHost, st));
  QST_S_HIP(hipMemcpyAsync(wb.data(), w_b, (size_t)R_b * 8, hipMemcpyDeviceToHost, st));
  // sum_{i,j} wq_i wx_j |<q_i|x_j>|^2 over the rows of Q (complex128) and of X (as given)
  auto gram = [&](const void* Q, const std::vector<double>& wq, const void* X, const std::vector<double>& wx,
                  double& acc) -> qst_status {
    std::vector<double> d((size_t)wq.size() * 2);
    acc = 0.0;
    for (size_t j = 0; j < wx.size(); ++j) {
      const void* xj = reinterpret_cast<const unsigned char*>(X) + j * D * cb;
      QST_S_HIP(qst::launch_dots(Q, (int)wq.size(), D, xj, c64, D, part.as<double>(), g1, dots.as<double>(), st));
      QST_S_HIP(hipMemcpyAsync(d.data(), dots.p, d.size() * 8, hipMemcpyDeviceToHost, st));
      QST_S_HIP(hipStreamSynchronize(st));
      for (size_t i = 0; i < wq.size(); ++i) acc += wq[i] * wx[j] * (d[2 * i] * d[2 * i] + d[2 * i + 1] * d[2 * i + 1]);
    }
    return QST_OK;
  };
  double aa = 0.0, ab = 0.0, bb = 0.0;
  QST_S_CALL(gram(qa.p, wa, atoms_a, wa, aa));
  QST_S_CALL(gram(qa.p, wa, atoms_b, wb, ab));
  QST_S_CALL(gram(qb.p, wb, atoms_b, wb, bb));
  if (!(bb > 0.0)) return qst_host_error(h, QST_ERR_NUMERIC, "reference state has zero norm");
  *out = std::sqrt(std::max(0.0, aa - 2.0 * ab + bb) / bb);
  return QST_OK;
}
