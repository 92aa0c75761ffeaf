/*
 * srtm.h -- parallel-in-time filtering and smoothing of linear Gaussian state-space
 * models with slow-rate integrated measurements (SRTM), on one AMD Instinct MI355X
 * (gfx950).
 *
 * Method: Yaghoobi & Sarkka, "Parallel state estimation for systems with integrated
 * measurements", arXiv 2410.00627. The problem is the one stated in Sec. III
 * (eq. original-linear-SSM and eq. dual-rate-ssm1); the plain entry points take it without
 * inputs (B = 0), the *_inputs ones with known inputs B u_{t-1} added to the dynamics:
 *
 *     x_t = F x_{t-1} + w_{t-1},        w ~ N(0, Q)          (F is the paper's A)
 *     y_k = (H / L) sum_{i=1..L} x_{k,i} + v_k,  v ~ N(0, R)  (H is the paper's C)
 *     x_0 ~ N(m0, P0);  window k = 1..N holds fast states x_{k,1..L}, i.e. fast times
 *     (k-1)L+1 .. kL; x_0 belongs to no window.
 *
 * srtm_filter returns p(x_{k,i} | y_{1:k}) (Sec. III-B, eq. update-fast) and the slow-rate
 * filter p(x_{k,L} | y_{1:k}) (Sec. III-A); srtm_smooth returns p(x_{k,i} | y_{1:N})
 * (Sec. III-C, eq. seq-smoothing-all) and the smoother's slow state p(x_{k,1} | y_{1:N})
 * (eq. seq-smoothing-1). Both are computed with the associative scans of Sec. IV
 * (eq. op-filter forward, eq. op-smoother in reverse) followed by a per-window pass that
 * recovers the fast-rate states (Remarks fast-par-filter and parallel-fast-smoothing).
 *
 * Conventions for every entry point:
 *  - All array arguments are DEVICE pointers (hipMalloc'd or equivalent), row-major,
 *    contiguous, of one element type given by srtm_shape.dtype, aligned to 16 bytes.
 *  - Index [k-1][i-1] addresses window k, fast step i. Covariances are full nx x nx,
 *    exactly symmetric, and only marginal (diagonal-block) covariances are returned.
 *  - The caller owns every buffer. The library allocates nothing, keeps no pointer
 *    after a call returns and holds no global mutable state; calls are reentrant.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the default stream) and the
 *    call returns without synchronising. Buffers must stay alive until the stream
 *    reaches the end of the call. Results are bitwise deterministic for a given shape.
 *  - Argument errors are returned synchronously before anything is enqueued.
 *    Numerical failures are OR-ed into the device int32 *info (which the caller zeroes
 *    beforehand; may be NULL): SRTM_INFO_* bits below. Outputs are unspecified when
 *    *info != 0.
 */
#ifndef SRTM_H
#define SRTM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { SRTM_F32 = 0, SRTM_F64 = 1 } srtm_dtype;

typedef enum {
  SRTM_OK = 0,
  SRTM_E_NULL = 1,        /* a required pointer is NULL                                */
  SRTM_E_SHAPE = 2,       /* N < 1, L < 1, nx < 1 or ny < 1, or sizes overflow          */
  SRTM_E_DTYPE = 3,       /* dtype is neither SRTM_F32 nor SRTM_F64                     */
  SRTM_E_UNSUPPORTED = 4, /* (nx, ny) pair not compiled, or L / N above the limits      */
  SRTM_E_ALIGN = 5,       /* an array is not 16-byte aligned (workspace: 256 bytes)     */
  SRTM_E_WORKSPACE = 6,   /* workspace_bytes smaller than srtm_workspace_size()         */
  SRTM_E_HIP = 7,         /* a HIP runtime call (kernel launch, event record) failed    */
  SRTM_E_SCRATCH = 8      /* srtm_smooth_noalloc: the problem needs more workspace than
                             the library's fixed scratch (SRTM_NOALLOC_SCRATCH_BYTES)     */
} srtm_status;

/* Device-side numerical status bits (OR-ed into *info). */
#define SRTM_INFO_INNOVATION_NOT_PD 1 /* C_bar P C_bar^T + R_x (eq. m-h-k-l) not positive definite */
#define SRTM_INFO_COMBINE_SINGULAR 2  /* I + D_i J_j of eq. op-filter numerically singular          */
#define SRTM_INFO_PRED_SINGULAR 4     /* A P^f_{k,l} A^T + Q of eq. parallel-ak-smoothing singular  */
#define SRTM_INFO_NONFINITE 8         /* a non-finite value reached an output                       */

/* Problem shape. nx = state size, ny = measurement size, L = window length (the
 * paper's l), N = number of windows (slow steps), dtype = element type of every array. */
typedef struct {
  int32_t nx;
  int32_t ny;
  int32_t L;
  int32_t dtype;
  int64_t N;
} srtm_shape;

/* Limits of this build (L bounds the per-step constant tables held in LDS). */
#define SRTM_MAX_L 128
#define SRTM_MAX_N (1LL << 26)

/* Largest input size of the *_inputs entry points. */
#define SRTM_MAX_NU 4

/* Bytes of device workspace srtm_filter (smoother = 0) or srtm_smooth (smoother = 1)
 * needs for `shape`. Returns SRTM_OK and writes *bytes, or an argument error. */
srtm_status srtm_workspace_size(const srtm_shape* shape, int32_t smoother, size_t* bytes);

/* Nonzero when the (nx, ny) pair is compiled into this library. */
int32_t srtm_supported(int32_t nx, int32_t ny);

/* Filtering (Sec. III-A/B, parallel IMKF of Sec. IV).
 *  Inputs (required):  F [nx][nx], Q [nx][nx], H [ny][nx], R [ny][ny], m0 [nx],
 *                      P0 [nx][nx], y [N][ny]   (Q, R, P0 symmetric PSD; R + H-part PD)
 *  Outputs (each may be NULL to skip it):
 *      m_fast [N][L][nx], P_fast [N][L][nx][nx]  : p(x_{k,i} | y_{1:k})
 *      m_slow [N][nx],    P_slow [N][nx][nx]     : p(x_{k,L} | y_{1:k})
 *  workspace: device buffer of at least srtm_workspace_size(shape, 0) bytes. */
srtm_status srtm_filter(const srtm_shape* shape,
                        const void* F, const void* Q, const void* H, const void* R,
                        const void* m0, const void* P0, const void* y,
                        void* m_fast, void* P_fast, void* m_slow, void* P_slow,
                        void* workspace, size_t workspace_bytes, int32_t* info, void* stream);

/* Smoothing (Sec. III-C, parallel IMS of Sec. IV), same inputs as srtm_filter.
 *  Outputs (each may be NULL to skip it):
 *      ms_fast [N][L][nx], Ps_fast [N][L][nx][nx] : p(x_{k,i} | y_{1:N})
 *      ms_slow [N][nx],    Ps_slow [N][nx][nx]    : p(x_{k,1} | y_{1:N})
 *      mf_fast, Pf_fast, mf_slow, Pf_slow          : the filter outputs of srtm_filter
 *  workspace: device buffer of at least srtm_workspace_size(shape, 1) bytes. */
srtm_status srtm_smooth(const srtm_shape* shape,
                        const void* F, const void* Q, const void* H, const void* R,
                        const void* m0, const void* P0, const void* y,
                        void* ms_fast, void* Ps_fast, void* ms_slow, void* Ps_slow,
                        void* mf_fast, void* Pf_fast, void* mf_slow, void* Pf_slow,
                        void* workspace, size_t workspace_bytes, int32_t* info, void* stream);

/* Smoothing with the lag-one cross-covariances of consecutive fast states (Remark
 * cross-covariances; the second moments that EM updates and the gradient of the
 * log-likelihood need), same inputs as srtm_filter:
 *      Cs_fast [N][L][nx][nx] : Cov(x_{k,i}, x_{k,i-1} | y_{1:N}), i = 1..L, with x_{k,0} = x_{k-1,L}
 *                               (the last fast state of window k-1) and x_{1,0} = x_0 ~ N(m0, P0);
 *                               required (SRTM_E_NULL when NULL), 16-byte aligned.
 *      ms_fast, Ps_fast, ms_slow, Ps_slow      : as srtm_smooth, each may be NULL.
 *  Inside a window Cov(x_{k,i}, x_{k,i-1} | y_{1:k}) = F P^f_{k,i-1} + (F c_{i-1} - c_i) S_k^{-1} U_{k,i-1}^T
 *  (c_i, U_{k,i}: the noise and total cross-covariances of x_{k,i} with y_k) plus the smoother's
 *  correction through x_{k,L}; across a boundary it is P^s_{k,1} G^T with the one-step gain
 *  G = P F^T (F P F^T + Q)^{-1} of the filter state (m, P) of x_{k-1,L} (eq. seq-smoothing-all).
 *  Time-invariant model without inputs. Workspace: srtm_workspace_size(shape, 1) bytes. Numerical
 *  status bits as srtm_smooth (4 also when F P F^T + Q is singular). */
srtm_status srtm_smooth_lag1(const srtm_shape* shape,
                             const void* F, const void* Q, const void* H, const void* R,
                             const void* m0, const void* P0, const void* y,
                             void* ms_fast, void* Ps_fast, void* ms_slow, void* Ps_slow, void* Cs_fast,
                             void* workspace, size_t workspace_bytes, int32_t* info, void* stream);

/* The paper's sequential comparison method (Sec. V: sequential IMKF and IMS) on the same GPU:
 * one lane walks the windows forwards with the IMKF (eq. prediction, eq. m-h-k-l) and backwards
 * with the sequential SRTM smoother (eq. seq-smoothing-all, eq. seq-smoothing-1), writing the same
 * smoothed outputs as srtm_smooth (each may be NULL) with no associative scan. For measurement
 * against the parallel path; work and depth are O(N). Workspace: srtm_workspace_size(shape, 1)
 * bytes. Errors and info bits as srtm_smooth. */
srtm_status srtm_smooth_sequential(const srtm_shape* shape,
                                   const void* F, const void* Q, const void* H, const void* R,
                                   const void* m0, const void* P0, const void* y,
                                   void* ms_fast, void* Ps_fast, void* ms_slow, void* Ps_slow,
                                   void* workspace, size_t workspace_bytes, int32_t* info, void* stream);

/* Profiling variant of srtm_smooth: identical work, and additionally sets events[2j] to the
 * start and events[2j+1] to the end of the j-th kernel it enqueues, j = 0 ..
 * srtm_kernel_count(1) - 1 (taken by the kernel's dispatch, so each interval is that kernel's
 * execution). `events` holds caller-created hipEvent_t handles and n_events must be at least
 * 2 * srtm_kernel_count(1). For measurement only; not for graph capture. */
srtm_status srtm_smooth_profiled(const srtm_shape* shape,
                                 const void* F, const void* Q, const void* H, const void* R,
                                 const void* m0, const void* P0, const void* y,
                                 void* ms_fast, void* Ps_fast, void* ms_slow, void* Ps_slow,
                                 void* mf_fast, void* Pf_fast, void* mf_slow, void* Pf_slow,
                                 void* workspace, size_t workspace_bytes, int32_t* info,
                                 void* stream, void* const* events, int32_t n_events);

/* ------------------------------------------------------------------ no allocation
 * For callers that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, and harnesses that forbid hipMalloc. srtm_smooth_noalloc is srtm_smooth
 * (same kernels, same outputs, bitwise) with its workspace taken from a scratch array the
 * library holds in device memory, SRTM_NOALLOC_SCRATCH_BYTES per GPU, which each GPU the
 * call runs on keeps until the process ends. The call itself allocates nothing and makes
 * no hipMalloc / hipFree.
 *  - Device: the scratch of the CURRENT device (hipGetDevice) is used; `stream` must belong
 *    to that device. Its address is looked up once per device, on the first call there.
 *  - Limit: problems whose workspace, srtm_workspace_size(shape, 1), exceeds
 *    SRTM_NOALLOC_SCRATCH_BYTES return SRTM_E_SCRATCH before anything is enqueued (for
 *    nx = 4, ny = 2, L = 20 in float64 that is about 2^17 windows).
 *  - Sharing: every call on one GPU uses that GPU's one array, which keeps whatever the last
 *    call left there (nothing in it has to start at zero). Calls that overlap on one GPU
 *    (other streams, other host threads) RACE on the array: serialise them.
 *  - Arguments, outputs, errors and info bits as srtm_smooth; SRTM_E_HIP if the scratch
 *    address cannot be obtained. */
#define SRTM_NOALLOC_SCRATCH_BYTES (64u << 20)
srtm_status srtm_smooth_noalloc(const srtm_shape* shape,
                                const void* F, const void* Q, const void* H, const void* R,
                                const void* m0, const void* P0, const void* y,
                                void* ms_fast, void* Ps_fast, void* ms_slow, void* Ps_slow,
                                void* mf_fast, void* Pf_fast, void* mf_slow, void* Pf_slow,
                                int32_t* info, void* stream);

/* ------------------------------------------------------------------ known inputs
 * The model of eq. original-linear-SSM with its input term:
 *     x_t = F x_{t-1} + B u_{t-1} + w_{t-1},
 * so the input u_{k,i-1} of window k drives the fast state x_{k,i}. Over one window the
 * inputs add the deterministic response z_{k,i} = sum_{j=1..i} F^{i-j} B u_{k,j-1} to the
 * fast states, i.e. B_bar u_bar_k to the slow state equation (eq. h-k-l-2) and
 * (H / L) sum_i z_{k,i} to the measurement (eq. y-k-l-2); the smoother's prediction of
 * x_{k+1,1} (eq. seq-smoothing-all) gains B u_{k+1,0}. Covariances do not change.
 *  B: device [nx][nu];  u: device [N][L][nu], u[k-1][i-1] = u_{k,i-1} (both of the call's
 *  dtype, 16-byte aligned);  1 <= nu <= SRTM_MAX_NU;  reserved must be 0. */
typedef struct {
  const void* B;
  const void* u;
  int32_t nu;
  int32_t reserved;
} srtm_inputs;

/* Bytes of device workspace the *_inputs entry points need: srtm_workspace_size plus one
 * per-window record (N (nx + ny) scalars) of the measurement with the input response removed. */
srtm_status srtm_workspace_size_inputs(const srtm_shape* shape, int32_t smoother, size_t* bytes);

/* srtm_filter, srtm_smooth and srtm_loglik with known inputs (same outputs and errors; the
 * workspace is srtm_workspace_size_inputs(shape, 0) bytes for the filter and the
 * log-likelihood and srtm_workspace_size_inputs(shape, 1) for the smoother; `inputs` NULL or
 * with a NULL array -> SRTM_E_NULL, nu out of range or reserved != 0 -> SRTM_E_SHAPE). */
srtm_status srtm_filter_inputs(const srtm_shape* shape, const srtm_inputs* inputs,
                               const void* F, const void* Q, const void* H, const void* R,
                               const void* m0, const void* P0, const void* y,
                               void* m_fast, void* P_fast, void* m_slow, void* P_slow,
                               void* workspace, size_t workspace_bytes, int32_t* info, void* stream);
srtm_status srtm_smooth_inputs(const srtm_shape* shape, const srtm_inputs* inputs,
                               const void* F, const void* Q, const void* H, const void* R,
                               const void* m0, const void* P0, const void* y,
                               void* ms_fast, void* Ps_fast, void* ms_slow, void* Ps_slow,
                               void* mf_fast, void* Pf_fast, void* mf_slow, void* Pf_slow,
                               void* workspace, size_t workspace_bytes, int32_t* info, void* stream);
srtm_status srtm_loglik_inputs(const srtm_shape* shape, const srtm_inputs* inputs,
                               const void* F, const void* Q, const void* H, const void* R,
                               const void* m0, const void* P0, const void* y,
                               void* ll, void* workspace, size_t workspace_bytes, int32_t* info, void* stream);

/* ------------------------------------------------------------------ time-varying models
 * The model given per window: window k's F_k, Q_k drive its fast steps x_{k,1} .. x_{k,L}
 * (the step from x_{k-1,L} into x_{k,1} included) and H_k, R_k give its measurement y_k:
 *     x_{k,i} = F_k x_{k,i-1} + w,  w ~ N(0, Q_k)   (x_{k,0} = x_{k-1,L}),
 *     y_k = (H_k / L) sum_i x_{k,i} + v_k,  v_k ~ N(0, R_k).
 * Each window's slow-rate model (Sec. III-A, eq. h-k-l-2 and eq. y-k-l-2) and window filter
 * (Sec. III-B) are built from its own matrices, and the smoother's prediction of x_{k+1,1}
 * (eq. seq-smoothing-all) uses F_{k+1}, Q_{k+1}. The scans combine whole filter elements
 * (eq. op-filter), since the elements no longer share their matrices.
 *  F [N][nx][nx], Q [N][nx][nx], H [N][ny][nx], R [N][ny][ny]: device arrays of the dtype;
 *  m0, P0, y and all outputs as in srtm_filter / srtm_smooth. nx <= 4 (SRTM_E_UNSUPPORTED
 *  otherwise). Workspace: srtm_workspace_size_tv(shape, 0) bytes for the filter and
 *  srtm_workspace_size_tv(shape, 1) for the smoother (per-window constants included). */
srtm_status srtm_workspace_size_tv(const srtm_shape* shape, int32_t smoother, size_t* bytes);
srtm_status srtm_filter_tv(const srtm_shape* shape,
                           const void* F, const void* Q, const void* H, const void* R,
                           const void* m0, const void* P0, const void* y,
                           void* m_fast, void* P_fast, void* m_slow, void* P_slow,
                           void* workspace, size_t workspace_bytes, int32_t* info, void* stream);
srtm_status srtm_smooth_tv(const srtm_shape* shape,
                           const void* F, const void* Q, const void* H, const void* R,
                           const void* m0, const void* P0, const void* y,
                           void* ms_fast, void* Ps_fast, void* ms_slow, void* Ps_slow,
                           void* mf_fast, void* Pf_fast, void* mf_slow, void* Pf_slow,
                           void* workspace, size_t workspace_bytes, int32_t* info, void* stream);

/* ------------------------------------------------------------------ log-likelihood and gradient
 * Marginal log-likelihood of the measurements, log p(y_{1:N}) = sum_k log N(y_k; C_bar m, S_k)
 * with the slow-rate filter's one-step prediction of y_k (eq. m-h-k-l; the Gaussian elements
 * of Sec. IV drop their normalisers, so it is accumulated from the innovations), written to
 * ll[0]. Workspace: srtm_workspace_size(shape, 0) bytes. */
srtm_status srtm_loglik(const srtm_shape* shape,
                        const void* F, const void* Q, const void* H, const void* R,
                        const void* m0, const void* P0, const void* y,
                        void* ll, void* workspace, size_t workspace_bytes, int32_t* info, void* stream);

/* log p(y_{1:N}) and its gradient with respect to F (dF [nx][nx]), Q and R (dQ [nx][nx],
 * dR [ny][ny]: symmetric-matrix gradients G, i.e. a small symmetric change E of Q changes
 * ll by tr(G E)).
 * Computed by Fisher's identity: the expected gradient of the complete-data log-density
 * under the smoothing distribution, written with the process noise w = x_t - F x_{t-1} and the
 * measurement residual r_k = y_k - (H/L) sum_i x_{k,i}: dF = Q^{-1} sum E[w x_{t-1}^T],
 * dQ = Q^{-1} sum (E[w w^T] - Q) Q^{-1} / 2, dR = R^{-1} sum (E[r r^T] - R) R^{-1} / 2. Each summand
 * is formed per fast step in that centred form, in float64 for both element types, from the same
 * forward and reverse scans as srtm_smooth (recomputed per window rather than stored). Workspace:
 * srtm_workspace_size(shape, 1) bytes. All outputs are device arrays of the shape's dtype. */
srtm_status srtm_loglik_grad(const srtm_shape* shape,
                             const void* F, const void* Q, const void* H, const void* R,
                             const void* m0, const void* P0, const void* y,
                             void* ll, void* dF, void* dQ, void* dR,
                             void* workspace, size_t workspace_bytes, int32_t* info, void* stream);

/* srtm_loglik_grad with known inputs (srtm_inputs; the same outputs, errors and centred noise
 * form). The fast-step smoothed means then carry the input response z_{k,i} of the input
 * section; the noise w = x_t - F x_{t-1} - B u_{t-1} and the measurement residual keep their
 * statistics, with the innovations taken against y_k minus the inputs' part. The gradient is with
 * respect to F, Q and R (B and u are given). Workspace: srtm_workspace_size_inputs(shape, 1). */
srtm_status srtm_loglik_grad_inputs(const srtm_shape* shape, const srtm_inputs* inputs,
                                    const void* F, const void* Q, const void* H, const void* R,
                                    const void* m0, const void* P0, const void* y,
                                    void* ll, void* dF, void* dQ, void* dR,
                                    void* workspace, size_t workspace_bytes, int32_t* info, void* stream);

/* ------------------------------------------------------------------ many sequences
 * One sequence of a batch: its own model (F, Q, H, R, m0, P0), measurements y [N][ny],
 * window length L and output arrays (each may be NULL), all DEVICE pointers of the batch's
 * dtype with the layouts of srtm_smooth. The sequences of a batch are independent problems
 * (each is the problem of Sec. III); they share only nx, ny and the dtype. */
typedef struct {
  const void *F, *Q, *H, *R, *m0, *P0, *y;
  void *ms_fast, *Ps_fast, *ms_slow, *Ps_slow;
  int64_t N;
  int32_t L;
  int32_t reserved; /* must be 0 */
} srtm_seq;

/* Plans a batch on the host. Validates every sequence (as srtm_smooth would), then returns
 * in *table_size the bytes of the batch table, in *workspace_size the device workspace the
 * batch needs, in *ntiles the number of 256-window tiles over all sequences and in *max_L
 * the largest window length. When `table` is not NULL and table_bytes >= *table_size, it
 * also writes the table there (host memory): per sequence a descriptor with its pointers
 * and its place in the workspace, then the sequence index of every tile. The caller copies
 * the table unchanged to device memory (16-byte aligned) before srtm_smooth_batch. Any
 * output pointer may be NULL (other outputs are written as usual). */
srtm_status srtm_batch_plan(int32_t nx, int32_t ny, int32_t dtype, const srtm_seq* seqs, int32_t nseq,
                            void* table, size_t table_bytes, size_t* table_size, size_t* workspace_size,
                            int64_t* ntiles, int32_t* max_L);

/* Smooths every sequence of a planned batch with one set of kernel launches: kernels over
 * sequences run one workgroup per sequence, kernels over tiles one workgroup per tile of
 * any sequence, so short and long sequences share the device. Each sequence's results are
 * bitwise equal to an srtm_smooth call on it alone. `table_host` is the plan's table and
 * `table_dev` its unchanged copy in device memory (16-byte aligned); the host copy is read
 * to check the workspace (at least the plan's size, 256-byte aligned) and to size the
 * launches. `info` holds one device int32 per sequence (zeroed by the caller; may be NULL).
 * Enqueues kernels only, so the call can be captured in a HIP graph. */
srtm_status srtm_smooth_batch(int32_t nx, int32_t ny, int32_t dtype, int32_t nseq, const void* table_host,
                              const void* table_dev, void* workspace, size_t workspace_bytes, int32_t* info,
                              void* stream);

/* srtm_loglik_grad for every sequence of a planned batch, in one set of launches. Here the
 * four output pointers of each srtm_seq given to srtm_batch_plan receive that sequence's
 * ll [1], dF [nx][nx], dQ [nx][nx] and dR [ny][ny] (all four required); everything else is as
 * in srtm_smooth_batch. */
srtm_status srtm_loglik_grad_batch(int32_t nx, int32_t ny, int32_t dtype, int32_t nseq, const void* table_host,
                                   const void* table_dev, void* workspace, size_t workspace_bytes, int32_t* info,
                                   void* stream);

/* ------------------------------------------------------------------ mixed batches
 * One sequence of a mixed batch: as srtm_seq, plus its own (nx, ny) (any supported pair),
 * optionally its known inputs (B [nx][nu], u [N][L][nu] as in srtm_inputs; NULL and nu = 0
 * without) or a per-window model (per_window = 1: F, Q, H, R laid out as in srtm_smooth_tv;
 * nx <= 4; no inputs then). Every pointer is a DEVICE pointer of the batch's dtype, 16-byte
 * aligned; any output may be NULL. Each sequence is the problem of Sec. III (with the input
 * term of srtm_inputs, or the per-window model of srtm_smooth_tv). */
typedef struct {
  int32_t nx, ny;
  int32_t L;
  int32_t per_window; /* 0 or 1 */
  int64_t N;
  const void *F, *Q, *H, *R, *m0, *P0, *y;
  const void *B, *u;
  int32_t nu;
  int32_t reserved; /* must be 0 */
  void *ms_fast, *Ps_fast, *ms_slow, *Ps_slow;
} srtm_seq_ex;

/* srtm_batch_plan for a mixed batch: validates every sequence (as srtm_smooth, srtm_smooth_inputs
 * or srtm_smooth_tv would), then returns the table and workspace sizes, the tile count and the
 * largest window length, and writes the table when `table` is large enough (same contract as
 * srtm_batch_plan; each descriptor also records its sequence's nx, ny and kind). */
srtm_status srtm_batch_plan_ex(int32_t dtype, const srtm_seq_ex* seqs, int32_t nseq, void* table,
                               size_t table_bytes, size_t* table_size, size_t* workspace_size, int64_t* ntiles,
                               int32_t* max_L);

/* Smooths every sequence of a mixed batch with ONE set of six kernel launches, whatever the mix
 * of (nx, ny) pairs and kinds: each workgroup dispatches on its own sequence's descriptor and
 * runs the same arithmetic on the same tiles as srtm_smooth (srtm_smooth_inputs, srtm_smooth_tv)
 * on that sequence alone. The launches size their registers and LDS for the largest pair
 * present, so a batch of one pair can be faster through srtm_smooth_batch. Arguments, checks
 * and info words as in srtm_smooth_batch (`table_host` and `table_dev` from srtm_batch_plan_ex).
 * Enqueues kernels only (capturable in a HIP graph). */
srtm_status srtm_smooth_batch_ex(int32_t dtype, int32_t nseq, const void* table_host, const void* table_dev,
                                 void* workspace, size_t workspace_bytes, int32_t* info, void* stream);

/* ------------------------------------------------------------------ HIP graphs
 * Thin wrappers over HIP stream capture so that a caller holding only streams can record a
 * sequence of calls (for instance srtm_smooth_batch_ex on several streams joined by events)
 * once and replay it. srtm_graph_begin starts capturing `stream` (relaxed mode; the legacy
 * default stream, NULL, cannot be captured: SRTM_E_NULL). srtm_graph_end ends the capture and
 * instantiates it into *exec (an opaque handle owned by the caller). srtm_graph_launch enqueues
 * one replay on `stream`; srtm_graph_destroy frees the handle. Captured calls must not allocate
 * or synchronise; every srtm_* launch entry point qualifies. Errors: SRTM_E_HIP with the HIP
 * error left for hipGetLastError. */
srtm_status srtm_graph_begin(void* stream);
srtm_status srtm_graph_end(void* stream, void** exec);
srtm_status srtm_graph_launch(void* exec, void* stream);
srtm_status srtm_graph_destroy(void* exec);

/* Number of kernels one srtm_filter (smoother = 0) or srtm_smooth (smoother = 1) call
 * enqueues, and the name of kernel j of that sequence (static string, or NULL). */
int32_t srtm_kernel_count(int32_t smoother);
const char* srtm_kernel_name(int32_t smoother, int32_t j);

/* Static text for a status code. */
const char* srtm_status_string(int32_t status);

/* Library version, major * 10000 + minor * 100 + patch. */
int32_t srtm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SRTM_H */
