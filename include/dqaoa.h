/*
 * dqaoa.h: C ABI of the MI355X (gfx950) QAOA state-vector library.
 *
 * The library simulates the QAOA ansatz of arXiv 2506.10531, Sec. IV, Eq. (2),
 *     |psi(theta)> = prod_{j=1..p} e^{-i H_X beta_j} e^{-i H gamma_j} |+>,
 * on the dense sub-QUBOs that the DQAOA decomposition step produces (Sec. V),
 * where H is diagonal with entries C(z) = z^T Q z (the QUBO energy of Eq. (1))
 * and H_X = -sum_i X_i.  Conventions shared by every entry point:
 *
 *   - bit i of the basis index z is variable i / qubit i (little endian);
 *   - layer j = 1 acts first on |+>;
 *   - the mixer factor is e^{+i beta sum_q X_q} (the paper's sign of H_X);
 *   - Q may be any dense real n x n matrix; C(z) = sum_ij Q_ij z_i z_j;
 *   - <C> = sum_z |psi(z)|^2 C(z) is the objective of Eq. (1).
 *
 * Memory: unless a comment says "host", every pointer is a DEVICE pointer on
 * the context's GPU, owned by the caller, and must stay valid until the work
 * queued on `stream` has finished.  Calls are stream-ordered and
 * asynchronous: they return after queueing work on `stream` (a hipStream_t;
 * NULL is the default stream).  Scratch memory (state vectors, checkpoints,
 * partial sums) belongs to the context, is charged against its HBM budget,
 * and is reused by the next call on the same context; the context orders
 * successive calls made on different streams.  A context must not be used
 * from two host threads at once.
 *
 * Errors: every function returns QAOA_OK (0), QAOA_PENDING (1, queue only) or
 * a negative QAOA_ERR_* code.  All argument checks happen on the host before
 * any device work is queued, so a rejected call has no side effect.
 * qaoa_last_error() returns a thread-local description of the last failure
 * on the calling thread (valid until that thread's next failing call).
 */
#ifndef DQAOA_H
#define DQAOA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qaoa_ctx qaoa_ctx;
typedef struct qaoa_queue qaoa_queue;
typedef void* qaoa_stream_t; /* a hipStream_t */

/* State precision. C128: complex128 amplitudes, FP64 arithmetic throughout.
 * C64: complex64 amplitudes and FP32 mixer arithmetic; the phase angle
 * gamma*C(z) is formed and range-reduced in FP64 before an FP32 sincos, and
 * <C>, the norm and gradients are accumulated in FP64. */
enum { QAOA_C128 = 0, QAOA_C64 = 1 };

enum {
  QAOA_OK = 0,
  QAOA_PENDING = 1,
  QAOA_ERR_INVALID_ARG = -1,
  QAOA_ERR_NO_DEVICE = -2,
  QAOA_ERR_OUT_OF_MEMORY = -3,
  QAOA_ERR_UNSUPPORTED = -4,
  QAOA_ERR_HIP = -5,
  QAOA_ERR_QUEUE_FULL = -6,
  QAOA_ERR_CANCELLED = -7,
  QAOA_ERR_TIMEOUT = -8,
  QAOA_ERR_NOT_FOUND = -9
};

#define QAOA_MAX_N 34      /* qubits per state (a 2^34 complex64 state is 128 GiB) */
#define QAOA_MAX_P 64      /* layers */
#define QAOA_DEVICE_NONE (-1)

/* Thread-local text of the last error on this thread ("" if none). */
const char* qaoa_last_error(void);
const char* qaoa_version(void);

/* Create a context on HIP device `device` with an HBM budget in bytes for
 * the context's scratch (0 = 90% of the device's free memory at creation).
 * device == QAOA_DEVICE_NONE makes a host-only context that plans and checks
 * arguments but runs nothing: its compute calls return QAOA_ERR_NO_DEVICE
 * after validation.  Errors: QAOA_ERR_NO_DEVICE (no such GPU),
 * QAOA_ERR_INVALID_ARG (out == NULL), QAOA_ERR_HIP. */
int qaoa_create(qaoa_ctx** out, int device, size_t hbm_budget);
/* Waits for the context's outstanding work and frees its scratch. */
int qaoa_destroy(qaoa_ctx* ctx);

/* <C> (Eq. (1) objective) of the Eq. (2) state for B problems x S parameter
 * sets each.
 *   Q       [B][n][n] FP64, row-major.
 *   gammas  [B][S][p] FP64;  betas [B][S][p] FP64.
 *   expect  [B][S] FP64 out.
 *   norm    [B][S] FP64 out, nullable: sum_z |psi(z)|^2.
 *   probs   [B][S][2^n] out, nullable: |psi(z)|^2 as FP64 (C128) or FP32
 *           (C64).
 * Errors: QAOA_ERR_INVALID_ARG (prec, B < 1, S < 1, n outside [1,
 * QAOA_MAX_N], p outside [1, QAOA_MAX_P], a NULL required pointer, or a size
 * whose byte count overflows), QAOA_ERR_OUT_OF_MEMORY (scratch beyond the
 * budget), QAOA_ERR_NO_DEVICE, QAOA_ERR_HIP. */
int qaoa_expect(qaoa_ctx* ctx, int prec, int B, int n, int p, int S,
                const double* Q, const double* gammas, const double* betas,
                double* expect, double* norm, void* probs,
                qaoa_stream_t stream);

/* qaoa_expect for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, results and errors as qaoa_expect, but the working memory
 * (state vectors, per-state pass tables, partial sums) comes from a fixed
 * device array of QAOA_NOALLOC_SCRATCH_BYTES that every GPU the library runs
 * on holds from qaoa_create until the process ends; the call itself makes no
 * hipMalloc, hipFree or other allocation and records no event.  Every call on
 * one GPU shares that array and leaves its contents behind (no call relies on
 * them: each writes every scratch word before reading it), so calls whose
 * work overlaps on one GPU race: issue them on one stream, or order them.
 * Errors as qaoa_expect; QAOA_ERR_OUT_OF_MEMORY when the B*S states, their
 * tables and partial sums exceed the array (e.g. one n = 24 or 16 n = 20
 * complex64 states fit). */
#define QAOA_NOALLOC_SCRATCH_BYTES (256ull << 20)
int qaoa_expect_noalloc(qaoa_ctx* ctx, int prec, int B, int n, int p, int S,
                        const double* Q, const double* gammas, const double* betas,
                        double* expect, double* norm, void* probs,
                        qaoa_stream_t stream);

/* The Eq. (2) state itself, psi [B][S][2^n] of interleaved (re, im) pairs:
 * FP64 pairs for C128, FP32 pairs for C64 (the library's state as computed).
 * expect/norm as in qaoa_expect (nullable).  Errors as qaoa_expect. */
int qaoa_state(qaoa_ctx* ctx, int prec, int B, int n, int p, int S,
               const double* Q, const double* gammas, const double* betas,
               void* psi, double* expect, double* norm, qaoa_stream_t stream);

/* Measurement of the Eq. (2) state (Sec. IV: the measured bit string is the
 * candidate solution): `shots` bit strings per problem, one parameter set
 * per problem.  Shot s draws u_s = (top 53 bits of SplitMix64 output s for
 * state `seed`) * 2^-53 and returns the smallest z whose running probability
 * sum exceeds u_s times the total probability.
 *   Q [B][n][n]; gammas, betas [B][p]  (FP64 in).
 *   z       [B][shots] uint64 out.
 *   cz      [B][shots] FP64 out, nullable: C(z) of each sample.
 *   best_z  [B] uint64 out: the sample of lowest C (ties: smallest z).
 *   best_c  [B] FP64 out: its C.
 *   expect  [B] FP64 out, nullable: <C> of the sampled state.
 * Errors as qaoa_expect, plus QAOA_ERR_INVALID_ARG for shots < 1. */
int qaoa_sample(qaoa_ctx* ctx, int prec, int B, int n, int p,
                const double* Q, const double* gammas, const double* betas,
                int shots, uint64_t seed, uint64_t* z, double* cz,
                uint64_t* best_z, double* best_c, double* expect,
                qaoa_stream_t stream);

/* d<C>/dgamma_j and d<C>/dbeta_j by the adjoint method: lambda = C psi_p is
 * carried back through the inverse layers, giving
 *   d<C>/dbeta_j  = -2 Im sum_q <lambda_j|X_q|psi_j>,
 *   d<C>/dgamma_j =  2 Im <lambda'_j|C|psi'_j>  (psi', lambda' after undoing
 *                                                 the mixer of layer j).
 * States of up to 13 (C64) or 12 (C128) qubits run in one launch with psi
 * and lambda in registers and use no scratch; larger states keep per-pass
 * checkpoints of psi in the context's scratch (charged to the budget).
 *   Q [B][n][n]; gammas, betas [B][S][p] (in).
 *   expect [B][S] out (nullable); dgamma, dbeta [B][S][p] out.
 * Errors as qaoa_expect. */
int qaoa_grad(qaoa_ctx* ctx, int prec, int B, int n, int p, int S,
              const double* Q, const double* gammas, const double* betas,
              double* expect, double* dgamma, double* dbeta,
              qaoa_stream_t stream);

/* Host-side plan of the state passes for (prec, n, p): how many HBM passes a
 * forward evaluation makes over each state, and the tile size in qubits.
 * `grad` != 0 plans the gradient's forward/backward sweeps instead.  Works on
 * a host-only context.  Errors: QAOA_ERR_INVALID_ARG. */
typedef struct {
  int sets;          /* disjoint qubit sets a layer's mixer is split into */
  int passes;        /* kernel passes over every state per evaluation */
  int state_reads;   /* full-state HBM reads per evaluation */
  int state_writes;  /* full-state HBM writes per evaluation */
  int tile_qubits;   /* qubits held in one LDS tile */
  int chunk_qubits;  /* low qubits kept contiguous in every tile */
  size_t scratch_bytes; /* context scratch this call needs for B*S states */
} qaoa_plan_info;
int qaoa_plan(qaoa_ctx* ctx, int prec, int B, int n, int p, int S, int grad,
              qaoa_plan_info* out);

/* The pass sequence behind qaoa_plan, one record of 10 ints per pass:
 * {set, tile_qubits k, contiguous low qubits c, first high tile bit a,
 *  first mixed tile qubit, lead layer (-1: none), first phase layer,
 *  last phase layer (first > last: none), flags, kernel (0: LDS tile,
 *  1/2: register tile, set 0 / the other sets)}.  (qaoa_expect and
 *  qaoa_state run states of up to 14 (C64) or 13 (C128) qubits, qaoa_grad
 *  up to 13 or 12, in one whole-state launch instead of the single pass
 *  listed.)  A pass applies the mixer
 * of the lead layer to its set, then for each phase layer j the phase of
 * layer j and the mixer of layer j on its set.  Tile qubits are global bits
 * [0, c) and [a, a + k - c) (all of [0, k) when c == k); the mixed tile
 * qubits are tile bits [first mixed, k).  Writes min(passes, max_passes)
 * records to host memory `out` and the pass count to *npass.  Errors:
 * QAOA_ERR_INVALID_ARG. */
int qaoa_plan_passes(qaoa_ctx* ctx, int prec, int n, int p, int grad,
                     int* out, int max_passes, int* npass);

/* Kernel timing on the stream each kernel is launched on: when enabled, the
 * context brackets every state-pass kernel launch with HIP events and
 * accumulates their durations.  qaoa_profile_read synchronises with the
 * recorded events and returns the number of pass launches and their total
 * time in milliseconds since the last reset.  A debugging and measurement
 * aid; it adds two events per launch. */
int qaoa_profile_enable(qaoa_ctx* ctx, int enable);
int qaoa_profile_read(qaoa_ctx* ctx, int reset, long long* launches,
                      double* total_ms, double* state_bytes);

/* ---------------------------------------------------------------------------
 * Solve queue: continuous batching of sub-QUBO solves (the "parallel
 * processing" step of the DQAOA workflow, Sec. V, served on one GPU).
 *
 * A request is one sub-QUBO solve: `evals` evaluations, each the exact <C>
 * and its adjoint gradient followed by one Adam step on (gamma, beta), then
 * <C> and `shots` samples at the final parameters.  A scheduler thread admits
 * pending requests in FIFO order while a slot is free and the request's
 * device bytes (its 2^n-amplitude state, checkpoints and adjoint state) fit
 * in the queue's HBM budget; every step it advances all admitted requests
 * together, one batched kernel sequence per distinct n and evaluation (up
 * to 16 evaluations per step, enqueued with two in flight; from the third on
 * the step ends early when a waiting request could be admitted), so
 * requests that arrive while others run share the GPU.  A request's result
 * does not depend on which other requests share its steps. */
typedef struct {
  int max_slots;        /* requests resident at once (>= 1) */
  int max_pending;      /* queued requests before qaoa_submit reports QUEUE_FULL */
  size_t hbm_budget;    /* device bytes for resident requests (0: half the context
                           budget, at most 80% of the memory free at creation) */
  int prec;             /* QAOA_C64 or QAOA_C128 */
  int p;                /* layers */
  int evals;            /* Adam steps per solve (>= 0) */
  int shots;            /* samples at the end (>= 1) */
  double lr, beta1, beta2, eps; /* Adam hyper-parameters */
  int batched;          /* 1: continuous batching; 0: one request at a time */
} qaoa_queue_opts;

typedef struct {
  int n;                /* qubits (variables of the sub-QUBO), 1..26 */
  const double* Q;      /* host [n][n] FP64; copied by qaoa_submit */
  const double* gamma0; /* host [p] initial gammas; copied */
  const double* beta0;  /* host [p] initial betas; copied */
  uint64_t seed;        /* sampling seed */
} qaoa_solve_req;

typedef struct {
  int status;           /* QAOA_OK, QAOA_ERR_CANCELLED or QAOA_ERR_HIP */
  int n;
  double gamma[QAOA_MAX_P];
  double beta[QAOA_MAX_P];
  double expect;        /* <C> at the final parameters */
  uint64_t best_z;      /* lowest-C sample (ties: smallest z) */
  double best_c;
  int64_t t_submit_ns, t_admit_ns, t_done_ns; /* CLOCK_MONOTONIC */
} qaoa_solve_result;

typedef struct {
  long long submitted, admitted, completed, cancelled, rejected;
  long long steps;      /* batched steps executed */
  int pending, active;  /* right now */
  size_t bytes_in_use;  /* device bytes held by resident requests */
  int peak_active;      /* most requests resident at once since creation */
  size_t peak_bytes;    /* most device bytes held by resident requests */
} qaoa_queue_stats;

int qaoa_queue_create(qaoa_ctx* ctx, const qaoa_queue_opts* opts,
                      qaoa_queue** out);
/* Stops and joins the scheduler, waits for the device work in flight and
 * frees the queue.  Requests not completed by then are dropped with it (their
 * tickets become invalid); no other call on the queue may be in progress or
 * follow (in particular no qaoa_wait on another thread). */
int qaoa_queue_destroy(qaoa_queue* q);
/* Thread-safe.  Copies Q and the initial parameters (host memory) before
 * returning.  Errors: QAOA_ERR_INVALID_ARG, QAOA_ERR_QUEUE_FULL (pending at
 * capacity: retry later), QAOA_ERR_OUT_OF_MEMORY (can never fit the budget). */
int qaoa_submit(qaoa_queue* q, const qaoa_solve_req* req, uint64_t* ticket);
/* QAOA_PENDING while queued or running; QAOA_OK once done (the result and,
 * if `samples` is non-NULL, host [shots] uint64 samples are copied out and
 * the ticket is released); QAOA_ERR_NOT_FOUND for an unknown ticket. */
int qaoa_poll(qaoa_queue* q, uint64_t ticket, qaoa_solve_result* out,
              uint64_t* samples);
/* As qaoa_poll, blocking up to timeout_ns (< 0: forever); QAOA_ERR_TIMEOUT. */
int qaoa_wait(qaoa_queue* q, uint64_t ticket, int64_t timeout_ns,
              qaoa_solve_result* out, uint64_t* samples);
/* Cancels a pending or running request; its result reports
 * QAOA_ERR_CANCELLED.  QAOA_ERR_NOT_FOUND if unknown or already finished. */
int qaoa_cancel(qaoa_queue* q, uint64_t ticket);
int qaoa_queue_get_stats(qaoa_queue* q, qaoa_queue_stats* out);

/* COBYLA-type optimisation of the QAOA parameters (Sec. IV: the paper's
 * variational loop, COBYLA from random values, there at p = 1) for B
 * independent problems Q (device [B][n][n]), problem b starting from
 * theta0[b] = (gamma_1..p, beta_1..p) (host [B][2p]) and minimising <C>
 * (Eq. (1)).  The unconstrained COBYLA steps: a simplex of 2p + 1 points,
 * the trust step to the minimiser of their linear interpolant within radius
 * rho, geometry steps that keep the simplex well shaped, rho halved from
 * rhobeg down to rhoend when the model predicts poorly; at most maxfun
 * evaluations per problem.  Every round, the points of all running
 * optimisers are evaluated by one qaoa_expect call.  Outputs (host): theta
 * [B][2p] the best point, expect [B] <C> there, nfev [B] evaluations
 * (nullable), rounds [1] batched calls (nullable), trace [B][maxfun][2p + 1]
 * (nullable): record k of problem b is its k-th evaluated point followed by
 * the <C> found there (records from nfev[b] on are left untouched).
 * Requires rhobeg >= rhoend > 0, maxfun >= 1.  Blocking (synchronises
 * stream); allocates its device buffers for the call. */
int qaoa_cobyla(qaoa_ctx* ctx, int prec, int B, int n, int p, const double* Q,
                const double* theta0, double rhobeg, double rhoend, int maxfun,
                double* theta, double* expect, int* nfev, int* rounds,
                double* trace, qaoa_stream_t stream);

/* Sampled objective of a sampler-based QAOA (the measurement of Sec. IV):
 * out[b] = CVaR_alpha of the shot energies cz[b][0..shots) (device, FP64,
 * e.g. from qaoa_sample), the mean over the lowest alpha fraction of the
 * empirical distribution with the boundary shot weighted fractionally:
 *   ( sum_{k <= floor(a)} E_(k) + (a - floor(a)) E_(floor(a)+1) ) / a,
 *   a = alpha * shots, E_(1) <= ... <= E_(shots);
 * alpha = 1 is the shot mean.  1 <= B <= 65535, 1 <= shots <= 65536,
 * 0 < alpha <= 1. */
int qaoa_cvar(qaoa_ctx* ctx, int B, int shots, const double* cz, double alpha,
              double* out, qaoa_stream_t stream);

/* ---- DQAOA outer cycle (Sec. V) ------------------------------------------
 * The classical steps around the sub-QUBO solves, on the device, for one
 * dense N x N QUBO Q (device, row-major FP64) and a global 0/1 solution x
 * (device, one byte per variable, non-zero = 1; E(x) = x^T Q x, Eq. (1)).
 * 1 <= N <= 65536; windows hold 1 <= k <= min(N, 64) variables.  Device
 * buffers are caller-owned; calls are stream-ordered and use no context
 * scratch.  Fixed-order FP64 sums make every result reproducible. */

/* Impact factors (Sec. V-A-2): impact[i] = E(x with x_i flipped) - E(x),
 * from one pass over Q via g = (Q + Q^T) x: impact[i] = d_i (Q_ii + g_i -
 * 2 Q_ii x_i), d_i = 1 - 2 x_i.  field [N] receives g (required: it also
 * holds Q x in between); energy [1] receives E(x) (nullable); order [N]
 * receives the variables ranked by |impact| (largest first, ties to the
 * smaller index, NaN last), always a permutation of [0, N) (nullable). */
int qaoa_impact(qaoa_ctx* ctx, int N, const double* Q, const uint8_t* x,
                double* impact, double* field, int32_t* order, double* energy,
                qaoa_stream_t stream);

/* IFD windows (the decomposition algorithm of Sec. V-A-2): window t of m is
 * order[(t*stride + r) mod N], r < k, sorted ascending, into choices
 * [m][k] int32.  stride 1 is the algorithm as printed (overlapping
 * windows); stride k gives disjoint windows.  order must be a permutation
 * of [0, N) (as qaoa_impact writes it). */
int qaoa_ifd_choices(qaoa_ctx* ctx, int N, const int32_t* order, int m, int k,
                     int stride, int32_t* choices, qaoa_stream_t stream);

/* BFS / PFS windows (Sec. V-A-3), mode QAOA_DECOMP_BFS or QAOA_DECOMP_PFS:
 * variables i, j interact when Q_ij + Q_ji != 0; window t starts at
 * order[t mod N] and grows to k variables.  BFS expands the window's
 * variables first-in first-out, taking each one's unselected neighbours by
 * |Q_ij + Q_ji| (largest first); PFS takes the unselected variable of
 * largest |impact| that interacts with the window.  With no such variable
 * both continue from the unselected variable of largest |impact|.  Ties go
 * to the smaller index.  choices [m][k] int32, each window sorted
 * ascending.  impact and order as qaoa_impact writes them; N <= 16384. */
int qaoa_traversal_choices(qaoa_ctx* ctx, int N, const double* Q,
                           const double* impact, const int32_t* order,
                           int mode, int m, int k, int32_t* choices,
                           qaoa_stream_t stream);

/* Sub-QUBOs (Sec. V, first step): subq[t] = Q[S_t, S_t], [m][k][k] FP64,
 * with S_t = choices[t][0..k) (ascending and distinct; bit r of a sub-QUBO
 * basis index is variable choices[t][r]).  Random decomposition (Sec.
 * V-A-1) passes randomly drawn windows here.  An index outside [0, N) sets
 * its row and column to NaN. */
int qaoa_decompose(qaoa_ctx* ctx, int N, const double* Q, int m, int k,
                   const int32_t* choices, double* subq, qaoa_stream_t stream);

/* Aggregation (Sec. V, third step): for t = 0..m-1 in order, the variables
 * of window t take the bits of subsol[t] (bit r -> choices[t][r]); the
 * change is kept only if it lowers E strictly.  field and energy must hold
 * (Q + Q^T) x and E(x) on entry (qaoa_impact) and are kept current, x is
 * updated in place; accepted [m] int32 (nullable) gets 1 / 0, or -1 for a
 * window holding an index outside [0, N) (skipped). */
int qaoa_aggregate(qaoa_ctx* ctx, int N, const double* Q, uint8_t* x,
                   double* field, double* energy, int m, int k,
                   const int32_t* choices, const uint64_t* subsol,
                   int32_t* accepted, qaoa_stream_t stream);

/* Bytes of device workspace qaoa_dqaoa_cycle needs (0 for invalid sizes). */
size_t qaoa_cycle_workspace(int N, int m, int k);

enum { QAOA_DECOMP_GIVEN = 0, QAOA_DECOMP_IFD = 1, QAOA_DECOMP_BFS = 2, QAOA_DECOMP_PFS = 3 };

typedef struct {
  double decompose_ms;  /* impact factors, windows, sub-QUBO gather + copy */
  double solve_ms;      /* the m sub-QUBO solves on the queue */
  double aggregate_ms;  /* aggregation of the best samples */
  int accepted;         /* windows whose sub-solution was kept */
  double energy;        /* E(x) after the cycle */
} qaoa_cycle_stats;

/* One DQAOA cycle (Sec. V): windows from the impact factors of x (mode
 * QAOA_DECOMP_IFD, with stride; QAOA_DECOMP_BFS / _PFS, N <= 16384) or from
 * choices (device [m][k], mode QAOA_DECOMP_GIVEN, e.g. random windows); the
 * m sub-QUBOs solved on queue
 * q (k <= 22 qubits each; initial parameters gamma0/beta0 are host arrays
 * of the queue's p; request t samples with seed + t); their best samples
 * aggregated into x.  field and energy [1] (device) receive (Q + Q^T) x and
 * E(x), work is a device buffer of qaoa_cycle_workspace(N, m, k) bytes.
 * Blocks until done (host stats, nullable).  A failed solve cancels the
 * remaining requests and returns its error; x is then unchanged. */
int qaoa_dqaoa_cycle(qaoa_ctx* ctx, qaoa_queue* q, int N, const double* Q,
                     uint8_t* x, double* field, double* energy, int mode, int m,
                     int k, int stride, const int32_t* choices,
                     const double* gamma0, const double* beta0, uint64_t seed,
                     void* work, qaoa_cycle_stats* stats, qaoa_stream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* DQAOA_H */
