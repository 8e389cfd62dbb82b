/* Runs every entry point of the FP64 oracle on tiny 1D, 2D and 3D problems, for a build
 * with AddressSanitizer and UndefinedBehaviorSanitizer (test infrastructure: only the
 * sanitizer test builds and runs it). Exits non-zero on a failed call; the sanitizers
 * abort on a bad access or undefined behaviour. */
#include <complex.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;
typedef struct {
    int32_t ndim, integrator;
    int64_t n[3];
    double lo[3], hi[3];
    int64_t batch;
    double h, alpha, gamma, gnl, trap[3], sigma;
    uint64_t seed;
    uint32_t id_base, noise_substeps;
    const double* Vgrid;
    double sigma_V;
    const double* convK;
    int32_t basis, pad0;
} ora_problem;

void ora_dft(const cplx* in, cplx* out, int64_t n, int sign);
void ora_fft(cplx* x, int64_t n, int sign);
void ora_philox_batch(const uint32_t* ctr, int64_t count, uint64_t seed, uint32_t* out);
void ora_noise(const ora_problem* p, int64_t step, cplx* xi);
int ora_step(const ora_problem* p, cplx* psi, int64_t step_index);
int ora_step_dense(const ora_problem* p, cplx* psi, int64_t step_index);
void ora_diag(const ora_problem* p, const cplx* psi, double* out);
void ora_overlap(const ora_problem* p, const cplx* phi, const cplx* psi, cplx* out);
void ora_moments(const ora_problem* p, const cplx* psi, double* mean, double* var);
int ora_run(const ora_problem* p, cplx* psi, int64_t step0, int64_t nsteps, int64_t sample_every, double* diag,
            cplx* ckpt, int64_t ckpt_every);
int ora_tangent(const ora_problem* p, cplx* psi, cplx* dpsi, const double* dV, int64_t step0, int64_t nsteps);
int ora_adjoint(const ora_problem* p, const cplx* psi0, int64_t step0, int64_t nsteps, int64_t ckpt_every,
                const cplx* lamT, cplx* grad_psi0, double* grad_V);
int ora_apply_D(const ora_problem* p, cplx* f, int dense, int adjoint);
int ora_fft_nd(const ora_problem* p, cplx* f, int sign);
void ora_ck_tableau(double* out);
void ora_vnoise(const ora_problem* p, int64_t step, double* eta);
int ora_ck_step(const ora_problem* p, const cplx* psi, double h, cplx* out, double* err, int ip);
int ora_ark45(const ora_problem* p, cplx* psi, double t_span, double tol, int64_t max_attempts, double* h,
              int64_t* stats, double* h_log, int64_t log_cap, int ip);

static int fails = 0;
#define CHECK(x)                                             \
    do {                                                     \
        if ((x) != 0) {                                      \
            fprintf(stderr, "failed: %s\n", #x);             \
            fails++;                                         \
        }                                                    \
    } while (0)

static void exercise(int ndim, const int64_t* n, int64_t batch, int si) {
    ora_problem p;
    memset(&p, 0, sizeof(p));
    p.ndim = ndim;
    int64_t M = 1;
    for (int a = 0; a < 3; a++) {
        p.n[a] = a < ndim ? n[a] : 1;
        p.lo[a] = -3.0;
        p.hi[a] = 3.0;
        p.trap[a] = 1.0 + 0.1 * a;
        M *= p.n[a];
    }
    p.batch = batch;
    p.h = 1e-3;
    p.alpha = 0.5;
    p.gamma = 0.05;
    p.gnl = 2.0;
    p.sigma = 0.01;
    p.seed = 7;
    p.id_base = 3;
    p.integrator = si;          /* RK4IP, then the semi-implicit step with noise substeps */
    p.noise_substeps = si ? 4 : 0;
    const int64_t tot = batch * M;
    double* V = malloc(sizeof(double) * tot);
    cplx* psi = malloc(sizeof(cplx) * tot);
    cplx* dpsi = malloc(sizeof(cplx) * tot);
    cplx* lam = malloc(sizeof(cplx) * tot);
    cplx* g = malloc(sizeof(cplx) * tot);
    double* gV = malloc(sizeof(double) * tot);
    double* dV = malloc(sizeof(double) * tot);
    cplx* xi = malloc(sizeof(cplx) * tot);
    for (int64_t j = 0; j < tot; j++) {
        V[j] = 0.01 * (double)(j % 7);
        psi[j] = (1.0 + 0.1 * (double)(j % 5)) + I * 0.05 * (double)(j % 3);
        dpsi[j] = 0.01 * (double)(j % 4) - I * 0.02;
        lam[j] = 0.3 - I * 0.01 * (double)(j % 6);
        dV[j] = 0.001 * (double)(j % 9);
    }
    p.Vgrid = V;
    ora_noise(&p, 5, xi);
    CHECK(ora_step(&p, psi, 3));
    CHECK(ora_step_dense(&p, psi, 4));
    CHECK(ora_apply_D(&p, psi, 0, 0));
    CHECK(ora_apply_D(&p, psi, 1, 1));
    CHECK(ora_fft_nd(&p, xi, -1));
    double* diag = malloc(sizeof(double) * batch * 4 * 4);
    cplx* ckpt = malloc(sizeof(cplx) * tot * 3);
    CHECK(ora_run(&p, psi, 10, 7, 3, diag, ckpt, 3));
    ora_diag(&p, psi, diag);
    cplx* ov = malloc(sizeof(cplx) * batch);
    ora_overlap(&p, psi, psi, ov);
    double* mean = malloc(sizeof(double) * M);
    double* var = malloc(sizeof(double) * M);
    ora_moments(&p, psi, mean, var);
    if (!si) {
        CHECK(ora_tangent(&p, psi, dpsi, dV, 2, 3));
        CHECK(ora_adjoint(&p, psi, 1, 5, 2, lam, g, gV));
    } else if (ora_adjoint(&p, psi, 1, 5, 2, lam, g, gV) == 0) {
        fails++; /* the adjoint is of the RK4IP step only */
    }
    /* noise in the potential (every lattice) and the non-local potential (1D) */
    double* K = malloc(sizeof(double) * p.n[0]);
    for (int64_t d = 0; d < p.n[0]; d++) K[d] = 1.0 / (1.0 + (double)(d < p.n[0] / 2 ? d : p.n[0] - d));
    double* eta = malloc(sizeof(double) * tot);
    p.sigma_V = 0.2;
    if (ndim == 1) p.convK = K;
    ora_vnoise(&p, 4, eta);
    CHECK(ora_step(&p, psi, 5));
    CHECK(ora_step_dense(&p, psi, 6));
    CHECK(ora_run(&p, psi, 10, 4, 2, diag, ckpt, 3));
    if (ora_tangent(&p, psi, dpsi, dV, 2, 3) == 0 || ora_adjoint(&p, psi, 1, 5, 2, lam, g, gV) == 0) fails++;
    p.sigma_V = 0.0;
    p.convK = NULL;
    if (ndim == 1) {
        /* the cosine and sine bases of a half domain */
        for (int basis = 1; basis <= 2; basis++) {
            p.basis = basis;
            CHECK(ora_step(&p, psi, 7));
            CHECK(ora_run(&p, psi, 10, 3, 0, NULL, NULL, 0));
        }
        p.basis = 0;
    }
    free(K), free(eta);
    /* the adaptive integrator is deterministic: it refuses noise, then runs without */
    double* hs = malloc(sizeof(double) * batch);
    int64_t* stats = malloc(sizeof(int64_t) * batch * 2);
    double* hlog = malloc(sizeof(double) * batch * 8);
    double* err = malloc(sizeof(double) * batch);
    for (int64_t b = 0; b < batch; b++) hs[b] = 1e-3;
    if (ora_ark45(&p, psi, 0.01, 1e-6, 100, hs, stats, hlog, 8, 1) != -1) fails++;
    p.sigma = 0.0;
    CHECK(ora_ck_step(&p, psi, 2e-3, g, err, 1));
    CHECK(ora_ck_step(&p, psi, 2e-3, g, err, 0));
    CHECK(ora_ark45(&p, psi, 0.01, 1e-6, 100, hs, stats, hlog, 8, 1));
    CHECK(ora_ark45(&p, psi, 0.01, 1e-6, 100, hs, stats, NULL, 0, 0));
    free(hs), free(stats), free(hlog), free(err);
    free(V), free(psi), free(dpsi), free(lam), free(g), free(gV), free(dV), free(xi);
    free(diag), free(ckpt), free(ov), free(mean), free(var);
}

int main(void) {
    cplx a[16], b[16];
    for (int i = 0; i < 16; i++) a[i] = i + I * (16 - i);
    ora_dft(a, b, 16, -1);
    ora_fft(a, 16, +1);
    uint32_t ctr[8] = {1, 2, 3, 4, 5, 6, 7, 8}, out[8];
    ora_philox_batch(ctr, 2, 0x1234567890ull, out);
    double tab[48];
    ora_ck_tableau(tab);
    const int64_t n1[1] = {16}, n2[2] = {8, 16}, n3[3] = {8, 8, 16};
    for (int si = 0; si < 2; si++) {
        exercise(1, n1, 3, si);
        exercise(2, n2, 2, si);
        exercise(3, n3, 1, si);
    }
    if (fails) return 1;
    printf("oracle entry points ran clean\n");
    return 0;
}
