/*
 * qst.h -- C ABI of the MI355X (gfx950) hot path of rank-adaptive matrix-free
 * atomic quantum state tomography.
 *
 * Problem statement (paper, problem-formulation section): a state is a convex
 * combination of pure-state atoms, rho = sum_r alpha_r |psi_r><psi_r| with
 * alpha on the simplex (eq. atomic-density); it is measured with B Pauli strings
 * s_b in {X,Y,Z}^N, each a product basis rotation V_b = V_{s_b,1} (x) ... (x)
 * V_{s_b,N} followed by a computational-basis readout (numerical-test section,
 * Pauli design).  The library evaluates the descriptor-level measurement
 * actions of the matrix-free oracle calls (matrix-free section): the atomic
 * Born map (eq. atomic-born-map), the loss (eq. qst-loss), the likelihood
 * ratio (eq. likelihood-ratio-vector), the weight gradient (eq.
 * weight-gradient), the atom Wirtinger gradient (eq. atom-wirtinger-gradient)
 * and the matrix-free product G v (eq. negative-gradient-product); plus the
 * coefficient step with pruning (eqs. coefficient-update, truncation-map) and
 * the spectral refactorisation (eqs. density-proposal .. spectral-selection).
 *
 * Conventions (the paper leaves them open; these are the readings used):
 *   - Qubit j (0-based; qubit 0 is the leftmost Kronecker factor) is bit
 *     N-1-j of the amplitude index and of the outcome index u.
 *   - Pauli codes: X = 0, Y = 1, Z = 2.  V_Z = I, V_X = (1/sqrt2)[[1,1],[1,-1]],
 *     V_Y = (1/sqrt2)[[1,-i],[1,i]]; outcome bit 0 is the +1 eigenvector.
 *   - Probabilities, frequencies and sensitivities are PER SETTING: row b of
 *     p sums to one for unit atoms.  Losses act on the stacked vectors
 *     pi = p/B and pihat = f/B, so for cross-entropy
 *         L = -sum_{b,u} (f/B) log(p/B + eps),   g = dL/dp = -(f/B)/(p/B+eps)/B,
 *     and for least squares (not in the paper)
 *         L = 1/2 sum (p/B - f/B)^2,             g = (p - f)/B^2.
 *   - Gradients: atom_grad[r] = dL/dpsi_r^* = alpha_r sum_b V_b^dagger (g_b * V_b psi_r)
 *     (conjugate-Wirtinger form of eq. atom-wirtinger-gradient; for
 *     cross-entropy it equals -alpha_r G psi_r); weight_grad[r] = dL/dalpha_r
 *     = sum_{b,u} g_{b,u} |(V_b psi_r)_u|^2 (= -(A^T c)_r for cross-entropy).
 *   - Atoms and weights are used exactly as given: no renormalisation.
 *
 * Memory and ownership: every bulk array is a caller-owned DEVICE pointer
 * (row-major, densely packed, complex numbers interleaved re,im).  The
 * library owns only the handle's workspace, which it allocates in
 * qst_plan (or on first use) and frees in qst_destroy; it never frees or
 * keeps caller memory beyond a call.  When a larger shape outgrows the
 * workspace, a new one is allocated and the old one is kept until
 * qst_destroy, so graphs captured earlier stay valid.  All calls are
 * asynchronous on the handle's stream; results are valid after the stream
 * is synchronised.
 *
 * Graph capture: qst_forward, qst_backward and qst_reweight_simplex may be
 * captured once the workspace fits (qst_plan, or one eager call with the same
 * shapes); they then enqueue kernels only (no allocation, no host sync, no
 * memset nodes).  A captured graph reads the workspace, so graphs of one
 * handle must not be replayed concurrently with each other or with eager
 * calls on a different stream.
 *
 * Errors: every call returns a qst_status.  Arguments are validated before
 * anything is enqueued; on error nothing is enqueued and the handle's last
 * error message is set.  Invalid Pauli codes in device memory (values > 2)
 * cannot be seen by the host: kernels treat them as Z and raise a device
 * flag that the next call on the handle reports as QST_ERR_NUMERIC.
 * No C++ exception crosses this interface.  One handle per thread.
 */
#ifndef QST_H
#define QST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QST_OK = 0,
  QST_ERR_INVALID_ARG = 1, /* null pointer, bad enum, negative size            */
  QST_ERR_SHAPE = 2,       /* sizes outside the supported range               */
  QST_ERR_ALIGN = 3,       /* pointer not aligned to its element size         */
  QST_ERR_UNSUPPORTED = 4, /* valid request this build does not implement     */
  QST_ERR_DEVICE = 5,      /* HIP runtime error (message in qst_last_error)  */
  QST_ERR_OOM = 6,         /* workspace allocation failed                     */
  QST_ERR_NUMERIC = 7,     /* a kernel raised its device flag (bad code or table entry) */
  QST_ERR_CAPTURE = 8      /* would allocate while the stream is capturing    */
} qst_status;

typedef enum {
  QST_LOSS_CE = 0,  /* eps-stabilised cross-entropy (eq. qst-loss)     */
  QST_LOSS_LS = 1,  /* least squares on the stacked probabilities      */
  QST_LOSS_NONE = 2 /* no loss: qst_backward takes the caller's dL/dp   */
} qst_loss;

typedef enum {
  QST_PATH_AUTO = 0,          /* BUTTERFLY_F32                                        */
  QST_PATH_BUTTERFLY_F32 = 1, /* staged per-qubit butterflies, complex64 atoms, FP32   */
  QST_PATH_BUTTERFLY_F64 = 2, /* same kernels in FP64, complex128 atoms                */
  QST_PATH_PLAIN_F32 = 3,     /* one HBM pass per qubit (reference kernel for speedups) */
  QST_PATH_TILE_F16 = 4,      /* one HBM pass per 4-qubit group: 16x16 complex Kronecker
                                 tiles on the matrix cores, FP16 operands (scaled per
                                 16x16 block), FP32 accumulation; complex64 atoms        */
  QST_PATH_TILE_BF16 = 5,     /* the same with BF16 operands (high and low parts); tiles
                                 with FP32 operands are not offered: at the FP32 matrix
                                 rate they cost more than the FP32 butterflies           */
  QST_PATH_BUTTERFLY_BF16 = 6 /* staged butterflies in FP32 with the setting-batch
                                 intermediates stored in BF16: half their HBM traffic;
                                 complex64 atoms, error about 1e-3 (tolerance 1e-2)      */
} qst_path;

/* One independent tomography instance (the arguments of the paper's problem
 * statement: atoms, weights, descriptor-level settings, observed frequencies).
 *   n_qubits  N, 1..30 (D = 2^N), with R 2^N times the bytes of a complex amplitude
 *             below 4 GiB (one setting's vectors are addressed through one 32-bit buffer
 *             range: N <= 24 at R = 16, N <= 28 at R = 1).  The staged kernels split the
 *             index bits into a low pass (all R atoms of a chunk on chip, R 2^(low bits)
 *             <= 2^14) and tile passes of 2^14 amplitudes with at most 2^10 rows over the
 *             bits above it: one pass when there are at most ten such bits; else, with Pauli
 *             settings and dense frequencies, a low pass over N - 10 bits that takes the
 *             atoms in turn (N <= 24), otherwise a middle and a top pass (N up to the low
 *             bits + 20).  The plain and tile paths take N <= 20 and R <= 16
 *             (QST_ERR_UNSUPPORTED beyond).
 *   rank      R, 1..256 (the atom count R_t).  Any such R runs when N >= 14 (staged
 *             passes), when R 2^N <= 2^14 (the whole state of every atom in one
 *             work-group), and for N = 11..13 on the FP32 path with Pauli settings and
 *             dense frequencies (on chip, atoms in turn); other shapes (ranks above
 *             2^(14-N) below 14 qubits) return QST_ERR_UNSUPPORTED.
 *   n_settings B >= 1
 *   atoms     [R][D] complex64 (complex128 for QST_PATH_BUTTERFLY_F64), 8-byte
 *             (16-byte) aligned
 *   weights   [R] float64 (alpha)
 *   settings  [B][N] uint8 Pauli codes
 *   freqs     [B][D] float32 per-setting frequencies N_{b,u}/N_s; may be NULL when
 *             no loss is requested
 *   settings_per_batch  0: library default (or the autotuned value); otherwise the
 *             number of settings per batch of intermediate amplitudes (>= 1), which
 *             also keeps the instance out of multi-instance batches
 *   probs_base  NULL, or [B][D] base probabilities in the path's real type (float32;
 *             float64 for QST_PATH_BUTTERFLY_F64), 4- (8-) byte aligned: the
 *             instance then describes p = probs_base + sum_r alpha_r |V_b psi_r|^2
 *             (a fixed part plus its atoms), and the loss, the sensitivities and
 *             both gradients act on that p.  This is the response update of the
 *             atom step (eq. pi-update): p_t as base, the old and the new atom
 *             with weights -alpha_r and +alpha_r (see qst_atom_trial).  With
 *             negative weights p may round below zero by about one ulp of
 *             probs_base; eps of the cross-entropy should cover it.
 *   unitaries   NULL (Pauli settings), or [n_unitaries][2][2] complex128 device array
 *             (row-major, re,im interleaved: 8 doubles each, 8-byte aligned) for
 *             general local product measurements (the paper's descriptor-level
 *             measurement actions): a code c >= 3 applies unitaries[c - 3] to its
 *             qubit before the computational-basis readout.  Each entry must be
 *             unitary (checked in FP64: columns of unit norm and orthogonal to 1e-6);
 *             an entry that is not, and codes >= 3 + n_unitaries, act as the
 *             identity and raise the device flag (QST_ERR_NUMERIC from a later call).
 *             Supported on QST_PATH_BUTTERFLY_F32 (and AUTO), one 2x2 per qubit and
 *             setting instead of the Pauli butterflies.
 *   n_unitaries 1..253 when unitaries is given, else ignored
 *   freqs_rowptr  NULL: freqs is dense [B][D].  Otherwise the frequencies are sparse
 *             (CSR, for few shots per setting): freqs holds the freqs_nnz non-zero
 *             values, freqs_index [freqs_nnz] int32 their outcomes u (strictly
 *             ascending within a row, 0 <= u < D) and freqs_rowptr [B+1] int64 the
 *             row starts (freqs_rowptr[0] = 0, freqs_rowptr[B] = freqs_nnz), all on
 *             the device.  Outcomes outside a row hold zero.  Malformed index data
 *             cannot make a kernel read or write outside these arrays or its own
 *             buffers; out-of-range outcomes are dropped.                       */
typedef struct {
  int32_t n_qubits;
  int32_t rank;
  int32_t n_settings;
  int32_t settings_per_batch;
  const void* atoms;
  const double* weights;
  const uint8_t* settings;
  const float* freqs;
  const void* probs_base;
  const double* unitaries;
  const int64_t* freqs_rowptr;
  const int32_t* freqs_index;
  int64_t freqs_nnz;
  int32_t n_unitaries;
} qst_instance;

typedef struct qst_handle qst_handle;

/* Create a handle bound to HIP device `device` and stream `hip_stream` (a
 * hipStream_t; NULL = the null stream).  *out receives the handle. */
qst_status qst_create(int device, void* hip_stream, qst_handle** out);
/* Destroy a handle and free its workspace (waits for its stream first). */
qst_status qst_destroy(qst_handle* h);
/* Re-bind the handle to another stream of the same device. */
qst_status qst_set_stream(qst_handle* h, void* hip_stream);
/* Static text for a status code. */
const char* qst_status_string(qst_status s);
/* Message of the last error on this handle ("" if none); valid until the next call. */
const char* qst_last_error(const qst_handle* h);

/* Reserve workspace for these shapes; when `autotune` is non-zero, implementation choices are
 * timed on the handle's stream (this synchronises): for one instance, the kernels, batch size
 * and tile bits of its shape (qst_choice below); for several, the routing of the whole call
 * (which instances run atoms-looped or as fused slices), kept for calls with the same shapes.
 * Later calls with shapes that fit the reservation allocate nothing, so they may be captured
 * into a HIP graph.  Optional: the compute calls plan implicitly. */
qst_status qst_plan(qst_handle* h, const qst_instance* inst, int n_inst, qst_path path, int autotune);

/* Implementation choices for one instance shape (n_qubits, rank, n_settings rounded up to a
 * power of two, path): which kernels run it and with which batch and tile sizes.  qst_plan with
 * autotune times the candidates that apply to the shape on a slice of at most 256 of its
 * settings and keeps the fastest, in the handle and in a process-wide cache keyed by the GPU
 * architecture and the shape (a later handle on the same architecture reuses it without timing).
 * Every field 0 (-1 for kind) means the library default.  Different choices give results equal
 * to rounding (the sums over settings and layouts are associated differently); one choice always
 * gives the same bits. */
typedef struct {
  int32_t kind;                  /* -1 default, 0 staged / one-chunk kernels (setting batches through
                                    HBM), 1 atoms looped on chip (n = 11..14), 2 fused slices (all
                                    atoms of a setting in one work-group: R 2^n <= 2^14)      */
  int32_t settings_per_batch;    /* kind 0: settings per batch of intermediates               */
  int32_t tile_bits_fwd;         /* kind 0 with high bits: tile bits of the forward tile stage */
  int32_t tile_bits_adj;         /* ... and of the adjoint tile stage (11..14, shape permitting) */
  int32_t values_per_thread_log2;/* kind 1: 4 (n = 13, 14) or 5                               */
  int32_t w_row_bits;            /* kind 0 with high bits, two passes: the adjoint tile stage reads
                                    rows of the low stage's output 2^w_row_bits elements apart
                                    (tile columns..low bits; the low bits: plain [S][R][D] order) */
  int32_t x_row_bits;            /* ... and the forward tile stage writes its rows for the low
                                    stage 2^x_row_bits elements apart (likewise)               */
  int32_t tuned;                 /* out: 1 when the choice comes from qst_plan's timing        */
  double best_ms;                /* out: time of the chosen candidate on the timing slice      */
  double default_ms;             /* out: time of the library default on the same slice         */
} qst_choice;

/* Read (set = 0) or pin (set = 1) the choice for the shape of `inst` on `path`.  Reading a shape
 * without a choice returns the defaults (kind -1, tuned 0).  A pinned choice is used by every
 * later call on this handle with that shape; a kind that does not apply to a call's instance
 * (e.g. unaligned arrays, general settings) falls back to the default for that call. */
qst_status qst_plan_choice(qst_handle* h, const qst_instance* inst, qst_path path, int set, qst_choice* choice);

/* Forward map (eq. atomic-born-map) for n_inst instances.
 *   probs[i]  [B][D] per-setting probabilities (float32; float64 for the F64 path),
 *             or NULL (not materialised); `probs` itself may be NULL.
 *   loss      [n_inst] float64 device array or NULL; requires freqs and loss != NONE.
 * Outputs are overwritten. */
qst_status qst_forward(qst_handle* h, const qst_instance* inst, int n_inst, void* const* probs,
                       double* loss, qst_loss loss_kind, double eps, qst_path path);

/* Fused forward + adjoint: loss, weight gradient and atom gradient in one pass
 * over the settings (eqs. qst-loss, weight-gradient, atom-wirtinger-gradient).
 *   grad_p      NULL: g comes from `loss_kind` and freqs.  Otherwise grad_p[i] is the
 *               caller's dL/dp [B][D] (float32; float64 for the F64 path) and
 *               loss_kind must be QST_LOSS_NONE (autograd route).
 *   atom_grad   [i] -> [R][D] complex64 (complex128 for F64), overwritten.
 *   weight_grad [i] -> [R] float64, overwritten (entry may be NULL).
 *   loss        [n_inst] float64 or NULL.
 *   project_tangent  non-zero: atom_grad[r] <- (I - psi_r psi_r^*) atom_grad[r]
 *               (tangent space of the complex sphere, eq. atom-projected-descent-direction). */
qst_status qst_backward(qst_handle* h, const qst_instance* inst, int n_inst, const void* const* grad_p,
                        void* const* atom_grad, double* const* weight_grad, double* loss,
                        qst_loss loss_kind, double eps, int project_tangent, qst_path path);

/* qst_backward for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  Same arguments,
 * validation and results as qst_backward; it calls no allocating routine.  Instead of
 * the handle's workspace, the library's scratch (decoded settings, setting-batch
 * intermediates, partial sums) lives in one fixed device array of 64 MiB per GPU, which
 * the library holds from its first qst_create on that GPU until the process ends.
 *   - The settings-per-batch S is lowered until the call fits the 64 MiB (an instance's
 *     own settings_per_batch is kept as given); batches of small instances that do not
 *     fit run one instance at a time.  Results equal qst_backward's bit for bit when the
 *     batch sizes are the same, else to summation order.
 *   - A call that needs more (e.g. n=20 at R=16, one setting of which is 2 x 128 MiB)
 *     returns QST_ERR_SHAPE with the size it needs, before anything is enqueued.
 *   - Every call on one GPU shares that GPU's array, which keeps the last call's
 *     contents: calls that overlap in time on one GPU (other streams, other handles,
 *     concurrent graph replays) race and must be serialised by the caller.
 *   - Nothing has to start zeroed: every scratch entry a call reads was written by the
 *     same call first. */
qst_status qst_backward_static(qst_handle* h, const qst_instance* inst, int n_inst, const void* const* grad_p,
                               void* const* atom_grad, double* const* weight_grad, double* loss,
                               qst_loss loss_kind, double eps, int project_tangent, qst_path path);

/* Trial response of an atom step (update rules for the atom slots: eqs.
 * atom-trial and pi-update).  With atom r of `inst` replaced by psi_trial,
 *     p~ = p_t + alpha_r (a(psi_trial) - a(psi_r)),   a(psi)_{b,u} = |(V_b psi)_u|^2,
 * and the loss at p~ -- what the acceptance rule (eq. state-acceptance-rule)
 * compares -- without recomputing the other R-1 atoms.  The two one-atom
 * responses run as one two-atom instance with weights (alpha_r, -alpha_r) on
 * the base p_t: one pass at about 2/R of a full forward.
 *   r            atom index, 0 <= r < rank
 *   psi_trial    [D] complex64 (complex128 for F64) device vector, used as given
 *   probs_t      [B][D] current probabilities (as written by qst_forward for this
 *                instance; float32, float64 for F64), or NULL: p~ is then the
 *                increment alpha_r (a(psi_trial) - a(psi_r)) alone
 *   probs_trial  [B][D] output or NULL;  loss_trial: one float64 or NULL (needs freqs
 *                and loss_kind != NONE).  inst->probs_base must be NULL.
 * The pair of atoms and weights is staged in the handle's workspace by a copy
 * kernel, so the call is capturable once the workspace fits.  Neither output may
 * alias probs_t or the atoms. */
qst_status qst_atom_trial(qst_handle* h, const qst_instance* inst, int r, const void* psi_trial,
                          const void* probs_t, void* probs_trial, double* loss_trial, qst_loss loss_kind,
                          double eps, qst_path path);

/* Coefficient step with pruning (eqs. coefficient-update, truncation-map), FP64,
 * one work-group on the device (no allocation, capturable):
 *   beta = proj_simplex(alpha + eta_alpha * hvec);  keep = {r : beta_r > tau}
 *   (if empty, the first maximum);  alpha_out[0..R_out) = beta_keep / sum(beta_keep),
 *   alpha_out[R_out..R) = 0;  keep_idx[0..R_out) ascending;  *R_out on the device.
 * hvec is A^T c = -dL/dalpha.  R in 1..1024.  All pointers are device pointers. */
qst_status qst_reweight_simplex(qst_handle* h, const double* alpha, const double* hvec, int R,
                                double eta_alpha, double tau, double* alpha_out, int32_t* keep_idx,
                                int32_t* R_out);

/* Spectral refactorisation of one instance's current state (update rules for the
 * spectral slots; Theorem 1).  Lanczos on S = rho + eta_rho G, where
 * G = -sum_m (dL/dpi_m) E_m comes from the current state and freqs (eq.
 * density-proposal), with products S v = sum_r alpha_r psi_r <psi_r|v> + eta_rho G v
 * (eq. density-product); k = min(n_lanczos, D) steps from the start vector v0
 * with full re-orthogonalisation; the top L = min(L_max, k) Ritz pairs; for
 * s = 1..L the candidate P_tau(proj_{Delta_s}(lambda_1..s), Phi_s) (eq.
 * spectral-candidates) scored by the proximal surrogate (eq. proximal-surrogate)
 * without its constant ||S||^2/(2 eta_rho); s* = first minimiser.
 * Host-orchestrated (synchronises the stream; not capturable).
 *   v0          [D] complex128 device start vector (the random draw is an input)
 *   atoms_out   [L_max][D] complex64 (complex128 for F64): rows 0..R_out-1 hold the
 *               chosen candidate's atoms (Ritz vectors), the rest is zero
 *   weights_out [L_max] float64 (zeros beyond R_out);  R_out, s_star: one int32 each
 *   ritz_vals, ritz_resid, q_scores: [L_max] float64 (entries beyond L are zero)
 * All output pointers are device pointers. */
qst_status qst_refactor(qst_handle* h, const qst_instance* inst, qst_loss loss_kind, double eps,
                        double eta_rho, double mu, double tau, int L_max, int n_lanczos, const void* v0,
                        void* atoms_out, double* weights_out, int32_t* R_out, int32_t* s_star,
                        double* ritz_vals, double* ritz_resid, double* q_scores, qst_path path);

/* Parameters of the rank-adaptive iteration (Algorithm 1); the defaults of Table
 * sim-parameters in brackets. */
typedef struct {
  int32_t max_slots;     /* T: slots t = 0..T-1                                            */
  int32_t t_alpha;       /* [5]  coefficient slot when t % t_alpha == 0 (0: never)           */
  int32_t t_ref;         /* [50] spectral slot when t % t_ref == 0, tested first (0: never)  */
  int32_t n_grid;        /* [11] step grid {2^-j}, j = 0..n_grid-1, tried largest first     */
  int32_t rank_max;      /* [8]  R_max: capacity of the state and L of the Ritz step        */
  int32_t n_lanczos;     /* [30] Lanczos steps per spectral trial                           */
  int32_t stop_window;   /* [20] accepted updates over which delta is measured (0: off)     */
  int32_t loss_kind;     /* QST_LOSS_CE [paper] or QST_LOSS_LS                              */
  double stop_delta;     /* [1e-4] stop once the relative decrease over the window is below */
  double mu;             /* [1e-3] rank penalty of J = L + mu R (eq. fixed-rank-objective)   */
  double eps;            /* [1e-8] */
  double tau;            /* [1e-3] pruning threshold (eq. truncation-map)                   */
  double tau_acc;        /* [1e-10] acceptance margin (eq. state-acceptance-rule)           */
  int64_t oracle_budget; /* [1e5] stop once the oracle-call count reaches it (0: off)       */
} qst_solve_params;

/* The rank-adaptive iteration (Algorithm 1) on one instance, driven from the host
 * with every oracle call on the device:
 *   slot t: spectral when t % t_ref == 0 (eqs. density-proposal .. spectral-selection,
 *   through qst_refactor), else coefficient when t % t_alpha == 0 (eq.
 *   coefficient-update and the pruning map, qst_reweight_simplex), else an atom step
 *   on atom r_t = t mod R_t (eqs. atom-direction, atom-trial; the response by eq.
 *   pi-update, qst_atom_trial).  Each trial takes the step sizes of the grid from
 *   the largest down and the first that satisfies the acceptance rule (eq.
 *   state-acceptance-rule, J = L + mu R) is kept; otherwise the state stays.
 *   Stopping (Table sim-parameters): max_slots, the relative decrease of J over the
 *   last stop_window accepted updates below stop_delta, or the oracle budget.  One
 *   oracle call is counted per gradient product (G psi_r or A^T c), per trial
 *   response with its loss, and per Lanczos product G v (n_lanczos, at most D, per
 *   spectral trial).
 *   inst         the initial state X_0 (rank R_0 <= rank_max, unit atoms), settings
 *                and freqs (required); probs_base must be NULL
 *   v0s          [n_v0][D] complex128 device: Lanczos start vectors, spectral slot k
 *                uses v0s[k mod n_v0] (the random draws are inputs); may be NULL
 *                when t_ref == 0
 *   atoms_out    [rank_max][D] complex64 (complex128 for F64), device: the final
 *                atoms, zero rows beyond the final rank; weights_out [rank_max]
 *                float64, device (zeros beyond);  rank_out: HOST int32
 *   history      HOST [max_slots][6] float64 or NULL: per slot run (t, kind 0 spectral
 *                / 1 coefficient / 2 atom, J after the slot, R after, accepted 0/1,
 *                accepted grid index or -1)
 *   info         HOST int64[3] or NULL: slots run, oracle calls, stop reason (0 slots,
 *                1 delta, 2 budget)
 * Synchronises the stream (the acceptance tests read scalars), allocates its own
 * scratch (two [B][D] probability arrays, two state copies) and is not capturable. */
qst_status qst_solve(qst_handle* h, const qst_instance* inst, const qst_solve_params* prm, const void* v0s,
                     int n_v0, void* atoms_out, double* weights_out, int32_t* rank_out, double* history,
                     int64_t* info, qst_path path);

/* Relative Frobenius distance e = ||rho_a - rho_b||_F / ||rho_b||_F of two atomic
 * states (the error metric of the numerical-test section), in Gram form without
 * dense matrices: ||sum_r a_r |u_r><u_r| ||_F^2 = sum_{r,r'} a_r a_r' |<u_r|u_r'>|^2,
 * and likewise for the cross term.  atoms_a [R_a][D], atoms_b [R_b][D] complex64
 * (complex128 for F64) and weights float64 on the device; *out on the HOST.
 * Synchronises; allocates scratch of (R_a + R_b) complex128 rows. */
qst_status qst_state_error(qst_handle* h, int n_qubits, const void* atoms_a, const double* w_a, int R_a,
                           const void* atoms_b, const double* w_b, int R_b, double* out, qst_path path);

/* Per-stage timing of the hot path (measurement support; not needed for results).
 * qst_profile_enable(h, 1) brackets every kernel launch the handle makes with a pair
 * of HIP events on its stream, grouped by stage kind:
 *   0 descriptor decode, 1 high-bit tile stage (forward), 2 fused low-bit stage,
 *   3 high-bit tile stage (adjoint, gradient accumulation), 4 reductions and
 *   epilogues, 5 other (reweight, refactor helpers, reference path), 6 one whole G v
 *   product of qst_refactor (its stages are then not counted under 1..4), 7 the middle
 *   pass of the three-pass schedule (states with more than ten bits above the low stage).
 * qst_profile_read synchronises the stream and returns, for one kind, the number of
 * launches and their summed event-to-event milliseconds since the last reset
 * (reset != 0 clears every kind).  Enabling allocates events; launches made while
 * the stream is capturing are not bracketed. */
qst_status qst_profile_enable(qst_handle* h, int enable);
qst_status qst_profile_read(qst_handle* h, int kind, int64_t* launches, double* total_ms, int reset);

/* Library build information: a static string (architecture, version). */
const char* qst_build_info(void);

#ifdef __cplusplus
}
#endif

#endif /* QST_H */
