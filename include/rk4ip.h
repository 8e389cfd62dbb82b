/*
 * rk4ip.h -- C ABI of the MI355X (gfx950) RK4 interaction-picture step library.
 *
 * The library advances fields psi(x, t) of coupled nonlinear Schroedinger /
 * Gross-Pitaevskii type equations
 *
 *     d psi / dt = L psi + G(psi),   L(k) = -i alpha |k|^2 - gamma,
 *     G(psi)     = -i (V(x) + g_nl |psi|^2) psi + sigma xi(x, t),
 *
 * on periodic Fourier lattices (Dennis, Hope & Johnsson, arXiv:1204.4255: the
 * problem of Sec. 3.6 eq. (5) with the NLSE right-hand side of eq. (7) and the
 * dimensionless trap form of Sec. 4.1 eq. (9); additive Wiener noise of Sec. 3.5).
 * One step is the fixed-step fourth-order Runge-Kutta scheme (Sec. 3.5) in the
 * interaction picture (Sec. 3.6, eqs. (5)-(6)), with the picture origin at the step
 * midpoint so that only D = e^{L dt/2} is needed (Sec. 3.6, last paragraph):
 *
 *     a  = D psi_n,             k1 = D[dt G(psi_n)],
 *     k2 = dt G(a + k1/2),      k3 = dt G(a + k2/2),
 *     k4 = dt G(D(a + k3)),     psi_{n+1} = D(a + k1/6 + k2/3 + k3/3) + k4/6.
 *
 * D is applied per lattice axis (the tensor-product factorisation of Sec. 3.2):
 * a 1D FFT along the axis, a multiply by e^{L_a dt/2}, the inverse FFT.
 *
 * Also available (each described at its flag, field or entry point):
 *   - the semi-implicit step (RK4IP_FLAG_SEMI_IMPLICIT) and noise substeps that sample one
 *     Wiener path at several step sizes (rk4ip_problem.noise_substeps);
 *   - the adaptive Cash-Karp RK4(5) in the interaction picture, or the explicit
 *     comparison method, for 1D groups (rk4ip_ark45);
 *   - a real Wiener noise in the potential (sigma_V) and, on 1D groups, a non-local
 *     convolution potential (conv_K);
 *   - cosine and sine bases on 1D half domains (basis).
 *
 * Conventions shared by every entry point
 *   - Fields are complex64, interleaved (re, im) float pairs, in device memory owned
 *     by the caller. One instance is n[2] x n[1] x n[0] values with axis 0 (x)
 *     contiguous; instances of a group are consecutive and groups follow each other
 *     in the order given to rk4ip_plan.
 *   - Lattice: x_{a,j} = lo[a] + j (hi[a] - lo[a]) / n[a], j = 0..n[a]-1 (half-open
 *     periodic domain); k_{a,m} = 2 pi / (hi[a] - lo[a]) * (m < n[a]/2 ? m : m - n[a]).
 *   - V(x) = 1/2 sum_a trap[a] x_a^2 + V_grid[b][j] (V_grid may be NULL).
 *   - Noise: xi is complex, E|xi|^2 = 1/(dt dV), held constant over the four stages of
 *     a step (Stratonovich, piecewise constant). It is Philox4x32-10 (Salmon et al.,
 *     SC'11) with key (seed low word, seed high word) and counter
 *     (j>>1, id_base + b, step low word, step bits 32..55) for point j of instance b;
 *     words (r0,r1) feed point 2q and (r2,r3) point 2q+1 through Box-Muller with
 *     u1 = ((r>>8)+1) 2^-24 and u2 = (r>>8) 2^-24. Noise is a pure function of
 *     (seed, instance, step, point), so runs resume bit-exactly from any step.
 *   - All calls are asynchronous on the plan's stream unless stated otherwise. The
 *     library never allocates device memory: the plan keeps its tables and work fields
 *     in the caller's workspace, which must stay valid until rk4ip_destroy.
 *   - Every call returns RK4IP_OK (0) or a negative status; nothing aborts and no C++
 *     exception crosses the ABI. A plan is not thread-safe; distinct plans are
 *     independent.
 *   - Device buffers are bare pointers, checked for NULL only: each must hold at least
 *     the elements its call documents (a field holds every point of every instance of
 *     every group, in group order), or kernels read and write past its end. Callers
 *     that hold sized buffers (the Python binding does) check the sizes before the call.
 */
#ifndef RK4IP_H
#define RK4IP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    RK4IP_OK = 0,
    RK4IP_ERR_INVALID_ARG = -1,         /* null pointer, bad count, dt <= 0, unknown flag,
                                           noise_substeps not a power of two <= 1024 */
    RK4IP_ERR_UNSUPPORTED_SHAPE = -2,   /* n[a] not a power of two in [8, 4096] (1D) or
                                           [8, 1024] (2D/3D), more than 2^29 points per
                                           instance (e.g. 1024^3), ndim not 1..3 */
    RK4IP_ERR_WORKSPACE_TOO_SMALL = -3,
    RK4IP_ERR_HIP = -4,                 /* a HIP runtime call failed; see rk4ip_last_error */
    RK4IP_ERR_NONFINITE = -5,           /* a diagnostic found a NaN or Inf in a field */
    RK4IP_ERR_NOT_CAPTURABLE = -6,      /* graph capture or replay failed */
    RK4IP_ERR_NO_DEVICE = -7            /* no usable gfx950 device */
};

/* Plan flags */
#define RK4IP_FLAG_GRAPH     0x1u  /* replay the steady-state steps of a run from a hipGraph */
#define RK4IP_FLAG_AUTOTUNE  0x2u  /* time candidate tile schedules at plan time and keep the best */
#define RK4IP_FLAG_FUSE_1D   0x4u  /* 1D groups: run several steps per launch with the line kept on chip */
/* The FP64-transform precision form: the forward step's FFTs, propagator multiply and
 * delta add run in FP64 inside the kernels (fields stay complex64 in memory, the pointwise
 * RK4 arithmetic stays FP32; tables are computed in FP64 and kept in FP64). It removes
 * most of the FP32 transform rounding that accumulates over long runs whose fields carry
 * high-k content (noise). Radix-8 schedules only; 1D lines up to 2048 points. The adjoint
 * passes keep FP32 transforms (their recomputed forward steps use this form). */
#define RK4IP_FLAG_FP64_TRANSFORMS 0x8u
/* The semi-implicit integrator (Sec. 3.5, the semi-implicit method, in the same
 * interaction picture with its origin at the step midpoint) in place of RK4:
 *
 *     a = D psi_n,   m = a + (dt/2) G(m) by three fixed-point iterations from m = a,
 *     psi_{n+1} = D (2 m - a).
 *
 * Second order in dt for deterministic problems, strong order one with additive noise,
 * and one G evaluation per iteration instead of four stages: the integrator the paper
 * uses for strong convergence of stochastic problems. The noise xi of a step is the same
 * Stratonovich draw as for RK4 (see noise_substeps). rk4ip_adjoint does not support it
 * (RK4IP_ERR_INVALID_ARG). */
#define RK4IP_FLAG_SEMI_IMPLICIT 0x10u
/* One launch per pass kind over every 2D/3D group of the plan (many instances of uneven
 * lattice size, as in the multi-path runs of Sec. 4.6) instead of one per group: a work
 * list divides the launch's workgroups among the groups. Every group's tiles use one fixed
 * schedule (radix 8, 256 threads: 2048/n lines or columns), the same arithmetic as the
 * per-group launches with that schedule. Takes RK4IP steps with FP32 transforms on 2D/3D
 * groups whose axes all have 128 or 256 points, with n[0] >= 2048/n[a] for a >= 1, at most
 * 64 groups (else RK4IP_ERR_UNSUPPORTED_SHAPE); 1D groups run as usual. The adjoint keeps
 * per-group launches. */
#define RK4IP_FLAG_MERGE_GROUPS 0x20u

typedef struct rk4ip_plan_s* rk4ip_plan_t;

/* One group of same-shape instances (paths or problem instances). */
typedef struct {
    int32_t ndim;            /* 1, 2 or 3 */
    int32_t basis;           /* 0: Fourier (periodic). 1D only: 1 cosine, 2 sine basis of a half
                                domain (Sec. 3.1: even / odd boundary conditions at both ends),
                                on the cell centres x_j = lo + (j + 1/2)(hi - lo)/n with modes
                                cos / sin(k_m (x - lo)), k_m = pi m / (hi - lo) (cosine,
                                m = 0..n-1) or pi (m + 1) / (hi - lo) (sine). The step runs
                                through the n-point transform of the reordered line (n <= 4096;
                                Makhoul's cosine transform, the propagator pairing modes m and
                                n - m); in the FP64-transform form or with sigma_V on the even /
                                odd extension (2n points: 2n <= 2048 / 4096). Not with conv_K.
                                Plans holding such a group take rk4ip_step and rk4ip_run
                                without samples; the other entry points return
                                RK4IP_ERR_INVALID_ARG. */
    int64_t n[3];            /* points per axis, axis 0 = x (contiguous); unused axes = 1 */
    double lo[3], hi[3];     /* periodic domain [lo, hi) per axis */
    int64_t batch;           /* instances in this group, >= 1 */
    double dt;               /* time step, > 0, equal for all groups of a plan */
    double alpha;            /* kinetic coefficient: L(k) = -i alpha |k|^2 - gamma */
    double gamma;            /* uniform linear damping rate (>= 0) */
    double g_nl;             /* nonlinear coefficient */
    double trap[3];          /* harmonic potential 1/2 trap[a] x_a^2 */
    const float* V_grid;     /* device [batch][M] float extra potential, or NULL */
    double sigma;            /* additive noise amplitude (0 = deterministic) */
    uint64_t seed;           /* Philox key */
    uint32_t id_base;        /* Philox instance id of the first instance of this group */
    uint32_t noise_substeps; /* S: the noise of step s is the normalised sum of the draws of
                                steps s S ... s S + S - 1 of a run with step dt/S, so that runs
                                with dt and dt/S sample one Wiener path (strong convergence
                                tests, Sec. 3.5). A power of two up to 1024; 0 and 1 mean one
                                draw per step. */
    /* The potential's extra terms: G gains -i (sigma_V eta + V_c) psi. */
    double sigma_V;          /* real Wiener noise in the potential (the stochastics example,
                                Sec. 4): eta is a real per-point noise held over the step,
                                E eta^2 = 1/(dt dV), Philox with counter tag 3 in the top byte
                                of the last counter word (the real part of the complex normal),
                                noise substeps as for xi. >= 0; 0 = none. */
    const double* conv_K;    /* host [n[0]] or NULL (1D groups only, else
                                RK4IP_ERR_UNSUPPORTED_SHAPE): the non-local potential (the non-local
                                example, Sec. 4) V_c(x_i) = dV sum_j K(x_i - x_j) |psi_j|^2 on
                                the periodic line, with K[d] = K(d dx) for d < n/2 and
                                K((d - n) dx) above. Read only by rk4ip_plan (and
                                rk4ip_workspace_bytes), which keeps its transform. */
} rk4ip_problem;

/* Bytes of device workspace rk4ip_plan needs for these groups: the spectral tables
 * (per axis: e^{L_a dt/2} in the form (cos-1, sin) and the FFT twiddles), two complex64
 * work fields per lattice point, and the FP64 reduction partials. Returns 0 when the
 * description is invalid. */
size_t rk4ip_workspace_bytes(const rk4ip_problem* probs, int nprob, uint32_t flags);

/* Validate the groups, build the tables (FP64, stored FP32) into `workspace`, choose the
 * per-pass schedules and return a plan bound to `stream` (a hipStream_t, NULL = the
 * default stream). `workspace` is device memory of at least rk4ip_workspace_bytes
 * bytes, 256-byte aligned. Synchronises the stream once (table upload). */
int rk4ip_plan(const rk4ip_problem* probs, int nprob, void* workspace, size_t ws_bytes, void* stream,
               uint32_t flags, rk4ip_plan_t* out);

/* Rebind the plan to another stream (a hipStream_t). */
int rk4ip_set_stream(rk4ip_plan_t plan, void* stream);

/* One step of every instance (RK4IP, or the semi-implicit step for plans made with
 * RK4IP_FLAG_SEMI_IMPLICIT), in place on `psi` (device complex64). step_index
 * selects the noise counters. */
int rk4ip_step(rk4ip_plan_t plan, void* psi, int64_t step_index);

/* nsteps steps starting at step index step0, in place on psi.
 *   sample_every > 0 and diag != NULL: diag (device, FP64) receives
 *     [nsteps/sample_every + 1][ninst][4] = (N, E_kin, E_pot, E_int) of the states at
 *     relative steps 0, s, 2s, ... (see rk4ip_diagnostics).
 *   ckpt != NULL and ckpt_every > 0: ckpt (device complex64) receives
 *     [ceil(nsteps/ckpt_every)][total points], the states at relative steps
 *     0, M, 2M, ... < nsteps (the checkpoints rk4ip_adjoint reads). */
int rk4ip_run(rk4ip_plan_t plan, void* psi, int64_t step0, int64_t nsteps, int64_t sample_every, double* diag,
              void* ckpt, int64_t ckpt_every);

/* FP64 integrals of the field (Sec. 3.4 quadrature with the uniform weight dV of a
 * Fourier lattice) for every instance: out (device) [ninst][4] =
 *   N = dV sum |psi|^2,
 *   E_kin = alpha dV sum_a (1/n_a) sum_lines sum_k k_a^2 |F_a psi|^2 (Parseval per axis),
 *   E_pot = dV sum V |psi|^2,  E_int = dV sum (g_nl/2) |psi|^4.
 * Sums run in a fixed order, so results are bit-reproducible. A non-finite N sets the
 * plan's sticky NONFINITE status (read with rk4ip_status). */
int rk4ip_diagnostics(rk4ip_plan_t plan, const void* psi, double* out);

/* Overlap c_b = dV sum_j conj(phi_j) psi_bj in FP64 for every instance b of group
 * `group`; phi (device complex64) holds one target field of that group's shape.
 * out (device) receives [batch][2] = (Re c, Im c). */
int rk4ip_overlap(rk4ip_plan_t plan, int group, const void* phi, const void* psi, double* out);

/* Moments over the instances of group `group` (many paths, Sec. 3.5): per point, the
 * mean of |psi|^2 and the sample variance of |psi|^2 with the (P-1) divisor, FP64,
 * accumulated in instance order. mean and var are device [M] arrays. */
int rk4ip_moments(rk4ip_plan_t plan, int group, const void* psi, double* mean, double* var);

/* Device workspace bytes rk4ip_adjoint needs for checkpoint spacing ckpt_every. */
size_t rk4ip_adjoint_workspace_bytes(rk4ip_plan_t plan, int64_t ckpt_every);

/* Adaptive fourth-fifth order Runge-Kutta in the interaction picture (Sec. 3.5: the
 * adaptive Cash-Karp pair, deterministic only; Sec. 3.6: eq. (6)) over [0, t_span], in
 * place on psi, for plans whose groups are all 1D and noise-free (sigma = sigma_V = 0;
 * G may include the non-local potential conv_K). Each instance adapts
 * its own step. With the picture origin at the start of each step, stage i at
 * t_n + c_i h is Y_i = psi_n + sum_j a_ij k_j, k_i = e^{-L c_i h} h G(e^{L c_i h} Y_i);
 * the step keeps psi_{n+1} = e^{L h}(psi_n + sum_i b_i k_i) (fifth order) and estimates
 * its error as ||sum_i (b_i - b*_i) k_i|| / ||psi_n + sum_i b_i k_i|| (relative L2 over
 * the instance). A step is accepted when the estimate is at most tol; the next trial
 * step is h min(5, max(1/5, 0.9 (tol/err)^{1/5})); the last step is cut to end on t_span.
 *   h      device double [ninst]: in, the first trial step of each instance (> 0); out,
 *          the next trial step (pass it back to continue the run over another interval).
 *          h lives on the device, so it is not checked here: an instance whose trial
 *          step is not positive and finite takes no step (its field and h are left as
 *          they were, stats = {0, 0, t_span == 0}).
 *   stats  device int64 [ninst][3]: accepted steps, rejected steps, 1 if t_span was
 *          reached (0 when the instance used max_attempts trial steps first).
 *   h_log  device double [ninst][log_cap]: the accepted step sizes in order (entries past
 *          the accepted count are left as they were), or NULL with log_cap = 0.
 * Transforms are complex64 in every precision form; the propagator of each trial step is
 * formed per mode from an FP64 phase. Asynchronous; allocates nothing. Returns
 * RK4IP_ERR_UNSUPPORTED_SHAPE for a plan with a 2D or 3D group and RK4IP_ERR_INVALID_ARG
 * for a noisy group, tol <= 0, t_span < 0 or max_attempts < 1.
 *   explicit_L  0: the interaction picture (above). 1: the comparison method of Sec. 3.6,
 *          the same pair on eq. (5) with the linear part evaluated in every stage as a
 *          spectral derivative, k_i = h (L Y_i + G(Y_i)), L Y = F^{-1}[L(k) F Y], and
 *          psi_{n+1} = psi_n + sum_i b_i k_i (its stable step falls as 1/k_max^2). */
int rk4ip_ark45(rk4ip_plan_t plan, void* psi, double t_span, double tol, int64_t max_attempts, double* h,
                int64_t* stats, double* h_log, int64_t log_cap, int explicit_L);

/* Discrete adjoint of rk4ip_run over nsteps steps from step0 (not in the paper).
 * Given the checkpoints written by rk4ip_run (same step0, nsteps, ckpt_every) and
 * lambda_T = dLoss/dRe psi_T + i dLoss/dIm psi_T (device complex64), writes
 * grad_psi0 (device complex64, same convention) and, if grad_V != NULL, adds nothing
 * but overwrites grad_V (device float [ninst][M]) with dLoss/dV_grid. Each segment of
 * ckpt_every steps is recomputed from its checkpoint into adj_ws and walked
 * backwards; V gradients accumulate in FP64. The recomputed states go straight into
 * their slots of adj_ws (one copy per segment, of its checkpoint). With RK4IP_FLAG_GRAPH a
 * whole segment is replayed from two hipGraphs (recompute, backward walk), recorded once
 * per adj_ws address and ckpt_every, so callers that reuse adj_ws replay them. Plans made
 * with RK4IP_FLAG_SEMI_IMPLICIT return RK4IP_ERR_INVALID_ARG (the adjoint is that of the
 * RK4IP step). */
int rk4ip_adjoint(rk4ip_plan_t plan, const void* ckpt, int64_t step0, int64_t nsteps, int64_t ckpt_every,
                  const void* lambda_T, void* grad_psi0, float* grad_V, void* adj_ws, size_t adj_ws_bytes);

/* Wait for the plan's stream and return the sticky status: RK4IP_OK,
 * RK4IP_ERR_NONFINITE (a diagnostic saw NaN/Inf) or RK4IP_ERR_HIP. Clears it. */
int rk4ip_status(rk4ip_plan_t plan);

/* Release the plan's host state (the workspace stays the caller's). Waits for the
 * plan's stream first. */
int rk4ip_destroy(rk4ip_plan_t plan);

/* Static description of a status code. */
const char* rk4ip_strerror(int status);

/* Last error message recorded on a plan (never NULL; "" when none). */
const char* rk4ip_last_error(rk4ip_plan_t plan);

/* Number of kernel pass kinds of group `group`, or a negative status: 1 for a 1D group
 * (the whole step in one launch); 4 for 2D (FIRST x, LF y, XF x, LAST2 x) and 6 for 3D
 * (FIRST x, D2 y, LF z, D2 y, XF x, LAST2 x). A run of n steps on a 2D/3D group launches
 * FIRST once, the middle passes n times, XF n - 1 times (it ends one step and starts the
 * next) and LAST2 once. */
int rk4ip_num_passes(rk4ip_plan_t plan, int group);

/* Name of pass `pass` of group `group` in the order above: kind, axis, length and tile
 * (for logs and profiles), or NULL if out of range. */
const char* rk4ip_schedule(rk4ip_plan_t plan, int group, int pass);

/* Per-pass timing with HIP events (tracing aid, off by default). While enabled, every
 * kernel pass that rk4ip_step/rk4ip_run enqueue outside a graph is bracketed by an event
 * pair on the plan's stream; enabling resets the counters. */
int rk4ip_profile(rk4ip_plan_t plan, int enable);

/* Wait for the plan's stream and return, for pass `pass` of group `group`, how many
 * launches were timed and their mean duration in milliseconds. */
int rk4ip_profile_read(rk4ip_plan_t plan, int group, int pass, int64_t* count, double* mean_ms);

/* ---- one step without a plan or a workspace --------------------------------------- */

/* For callers that cannot allocate device memory (code under stream capture, serving
 * loops, harnesses that forbid hipMalloc): one step of every instance, in place on psi,
 * exactly the step rk4ip_step makes on a plan built with flags 0 (RK4IP, FP32 transforms,
 * default tile schedules), without a plan or a caller workspace. The tables (computed on
 * the device in FP64 with the same expressions as rk4ip_plan's) and the work fields live in
 * a static device buffer of RK4IP_NOALLOC_SCRATCH_BYTES that the library holds on every
 * GPU it runs on until the process ends; the call allocates nothing and is asynchronous on
 * `stream` (a hipStream_t, NULL = the default stream).
 *   - The buffer must hold the groups' tables, two complex64 work fields per point of the
 *     2D/3D groups and one per point of the 1D Fourier groups (about 16 B per lattice point
 *     plus the tables, so up to about 4 million points): larger problems return
 *     RK4IP_ERR_WORKSPACE_TOO_SMALL (rk4ip_workspace_bytes(probs, nprob, 0) is the size
 *     needed).
 *   - At most 16 groups (RK4IP_ERR_INVALID_ARG); no non-local potential (conv_K: its table
 *     is a host-side transform; RK4IP_ERR_INVALID_ARG). Other arguments are checked as by
 *     rk4ip_plan; RK4IP_ERR_NO_DEVICE when the current device is not a gfx950.
 *   - Every call on one GPU shares that GPU's buffer and overwrites it: calls that overlap
 *     on one GPU (on different streams, or from different threads) race and must be
 *     serialised by the caller. Nothing in the buffer needs to start at zero. */
#define RK4IP_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int rk4ip_step_noalloc(const rk4ip_problem* probs, int nprob, void* psi, int64_t step_index, void* stream);

/* ---- test entry points (device pointers, asynchronous on `stream`) -------------- */

/* Philox4x32-10 words for n counters: ctr [n][4] uint32 in, out [n][4] uint32. */
int rk4ip_debug_philox(uint64_t seed, const uint32_t* ctr, int64_t n, uint32_t* out, void* stream);

/* The noise field xi (complex64) of every instance of group `group` at step `step`,
 * [batch][M]. */
int rk4ip_debug_noise(rk4ip_plan_t plan, int group, int64_t step, void* xi);

/* Unnormalised 1D FFTs (sign -1 forward, +1 inverse) of `nlines` contiguous complex64
 * lines of length n[axis] of group `group`, with the library's device FFT engine and
 * that axis's twiddle table. in and out are device [nlines][n]; out may equal in. */
int rk4ip_debug_fft(rk4ip_plan_t plan, int group, int axis, const void* in, void* out, int64_t nlines, int sign);

/* D = e^{L dt/2} (adjoint != 0: its transpose e^{conj(L) dt/2}) applied in place to
 * every instance of psi, through the same axis passes the step uses. */
int rk4ip_debug_apply_D(rk4ip_plan_t plan, void* psi, int adjoint);

#ifdef __cplusplus
}
#endif

#endif /* RK4IP_H */
