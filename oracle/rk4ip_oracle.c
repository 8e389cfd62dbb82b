/*
 * rk4ip_oracle.c -- double-precision CPU oracle for the RK4 interaction-picture step.
 *
 * TEST INFRASTRUCTURE. This file is the slow, plain reference that the HIP library is
 * checked against. Only the test suite, the smoke check and the benchmark's CPU-baseline
 * leg may load it. It shares no source, header, table or helper with the HIP library.
 *
 * Method (Dennis, Hope & Johnsson, "XMDS2: Fast, scalable simulation of coupled
 * stochastic partial differential equations", arXiv:1204.4255):
 *   - Fourier spectral representation on a periodic tensor-product lattice
 *     (Sec. 3.1, eq. (1); Fourier basis e^{i k_n x}).
 *   - Transforms between spatial and spectral representations are FFTs, factorised
 *     per dimension over the tensor-product lattice (Sec. 3.2).
 *   - Method of lines with the fixed-step fourth-order Runge-Kutta scheme (Sec. 3.5).
 *   - Interaction picture (Sec. 3.6, eqs. (5)-(6)): f~ = e^{-L t} f with L local in the
 *     spectral basis; for fixed steps only e^{+-L dt/2} is ever needed.
 *   - Nonlinear Schroedinger / Gross-Pitaevskii right-hand side (Sec. 3.6 eq. (7),
 *     Sec. 4.1 eq. (9)), kinetic term diagonal in k (eq. (8)).
 *   - Wiener noise in Stratonovich form (Sec. 3.5); many independent paths (Sec. 3.5,
 *     Sec. 4.6).
 *   - Integrals over the lattice by quadrature with uniform weights (Sec. 3.4).
 *
 * Readings where the paper is silent (each one is also listed in the design notes):
 *   R1  The RK4IP variant: the interaction-picture origin of step n is the midpoint
 *       t_n + h/2, so D = e^{L h/2} is the only exponential used (Sec. 3.6, last
 *       paragraph on fixed steps). Classic RK4 on eq. (6) then gives
 *         a  = D psi_n,            k1 = D[h G(psi_n)],
 *         k2 = h G(a + k1/2),      k3 = h G(a + k2/2),
 *         k4 = h G(D(a + k3)),     psi_{n+1} = D(a + k1/6 + k2/3 + k3/3) + k4/6.
 *   R2  L(k) = -i alpha |k|^2 - gamma (kinetic term of eq. (8) plus uniform damping).
 *   R3  G(phi) = -i (V + g |phi|^2) phi + sigma xi, V = 1/2 sum_a trap_a x_a^2 + Vgrid.
 *   R4  xi is complex, circular, held constant over the four stages of a step
 *       (Stratonovich, piecewise constant), E|xi|^2 = 1/(h dV). It is generated from
 *       Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) keyed by the seed, with
 *       counter (j>>1, instance id, step low word, tag<<24 | step high bits);
 *       words (r0,r1) feed point 2q and (r2,r3) point 2q+1 through Box-Muller with
 *       u1 = ((r>>8)+1) 2^-24 in (0,1], u2 = (r>>8) 2^-24 in [0,1).
 *   R5  Lattice x_{a,j} = lo_a + j dx_a, dx_a = (hi_a - lo_a)/n_a, half-open domain;
 *       k_{a,m} = 2 pi / (hi_a - lo_a) * (m < n_a/2 ? m : m - n_a).
 *   R6  The semi-implicit method (Sec. 3.5, deterministic order 2, stochastic order 1)
 *       is the implicit midpoint rule solved by fixed-point iteration, here with three
 *       iterations and in the interaction picture with its origin at the midpoint, so
 *       that D = e^{L h/2} is again the only exponential:
 *         a = D psi_n;  m <- a + (h/2) G(m) three times, starting from m = a;
 *         psi_{n+1} = D(2 m - a).
 *   R7  Sampling one Wiener path with several step sizes (the strong-convergence test of
 *       Sec. 3.5): with S = 2^L substeps the noise of step n is the mean of the S draws of
 *       a run with step h/S at steps nS ... nS + S - 1, i.e. xi = (sum_s z_s / sqrt(S)) /
 *       sqrt(2 h dV) with z_s the complex normals of those finer steps.
 *   R8  The adaptive fourth-fifth order Runge-Kutta method (Sec. 3.5, deterministic only)
 *       is the embedded pair of Cash and Karp (ACM TOMS 16, 201, 1990) applied to eq. (6)
 *       with the picture origin at the start of each step, so stage i at t_n + c_i h is
 *         Y_i = psi_n + sum_j a_ij k_j,   k_i = e^{-L c_i h} h G(e^{L c_i h} Y_i),
 *       the step keeps the fifth-order result, psi_{n+1} = e^{L h}(psi_n + sum_i b_i k_i)
 *       (local extrapolation), and the error estimate of the step is the relative L2
 *       norm over the instance, in the picture frame, of the difference between the
 *       fifth- and fourth-order results: ||sum_i (b_i - b*_i) k_i|| / ||psi_n + sum_i b_i k_i||.
 *       The comparison method of Sec. 3.6 ("explicit") takes the same pair on eq. (5) with the
 *       linear part evaluated in the stages as a spectral derivative, k_i = h (L Y_i + G(Y_i)),
 *       L Y = F^{-1}[L(k) F Y], and psi_{n+1} = psi_n + sum_i b_i k_i.
 *   R10 Noise in the potential (the stochastics example, Sec. 4): G gains
 *       -i sigma_V eta psi with eta a real Wiener noise per lattice point, held over the
 *       step like xi, E eta^2 = 1/(h dV); it is the real part of the complex normal drawn
 *       with counter tag 3 (unit variance), summed over noise substeps as in R7, divided by
 *       sqrt(h dV).
 *   R11 A non-local potential (the non-local example, Sec. 4: a convolution with the
 *       density): G gains -i V_c psi with V_c(x_i) = dV sum_j K(x_i - x_j) |psi_j|^2 on the
 *       periodic lattice, the kernel given at lattice offsets, K[d] = K(d dx) for
 *       d < n/2 and K((d - n) dx) above (1D lattices).
 *   R12 Cosine and sine bases (Sec. 3.1: even and odd boundary conditions at both ends of
 *       a 1D domain): the lattice is cell-centred, x_j = lo + (j + 1/2) dx; the modes are
 *       cos(k_m (x - lo)) with k_m = pi m / L (m = 0..n-1) and sin(k_m (x - lo)) with
 *       k_m = pi (m + 1) / L; the transforms are the DCT-II / DST-II sums and their
 *       inverses (DCT-III / DST-III), so e^{L h/2} multiplies mode m by exp(L(k_m) h/2).
 *   R9  Step control (the paper gives none): a step is accepted when its error estimate is
 *       at most tol; either way the next trial step is h min(5, max(1/5, 0.9 (tol/err)^{1/5}))
 *       (5 when err = 0; 1/5 when err is not finite). A trial step that would pass the end
 *       of the interval is cut to end on it. Each instance adapts its own step.
 *
 * Memory layout: one instance is n[0]*n[1]*n[2] complex values with axis 0 (x)
 * contiguous; instances are concatenated. Unused axes have n = 1.
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

typedef struct {
    int32_t ndim;
    int32_t integrator; /* 0: RK4IP (R1); 1: semi-implicit in the interaction picture (R6) */
    int64_t n[3];
    double lo[3];
    double hi[3];
    int64_t batch;
    double h;
    double alpha;
    double gamma;
    double gnl;
    double trap[3];
    double sigma;
    uint64_t seed;
    uint32_t id_base;
    uint32_t noise_substeps; /* 0 or 1: one draw per step; 2^L: the sum of 2^L finer draws (R7) */
    const double* Vgrid; /* [batch][M] or NULL */
    double sigma_V;      /* real noise in the potential (R10) */
    const double* convK; /* [n] kernel of the non-local potential (R11), 1D, or NULL */
    int32_t basis;       /* 0 Fourier; 1 cosine, 2 sine (R12), 1D */
    int32_t pad0;
} ora_problem;

#define ORA_PI 3.14159265358979323846

static int64_t npts(const ora_problem* p) { return p->n[0] * p->n[1] * p->n[2]; }

static double dx_of(const ora_problem* p, int a) { return (p->hi[a] - p->lo[a]) / (double)p->n[a]; }

static double dV_of(const ora_problem* p) {
    double dv = 1.0;
    for (int a = 0; a < p->ndim; a++) dv *= dx_of(p, a);
    return dv;
}

/* Wavenumber of mode m on axis a (reading R5). */
static double k_of(const ora_problem* p, int a, int64_t m) {
    int64_t n = p->n[a];
    int64_t s = (m < n / 2) ? m : m - n;
    return 2.0 * ORA_PI / (p->hi[a] - p->lo[a]) * (double)s;
}

static void unflatten(const ora_problem* p, int64_t j, int64_t idx[3]) {
    idx[0] = j % p->n[0];
    idx[1] = (j / p->n[0]) % p->n[1];
    idx[2] = j / (p->n[0] * p->n[1]);
}

/* ------------------------------------------------------------------------------------
 * Discrete Fourier transform. Forward uses e^{-2 pi i j m / n}, the inverse e^{+...};
 * neither is normalised. Sec. 3.2: FFT along each dimension of the lattice.
 * ---------------------------------------------------------------------------------- */

/* Brute force O(n^2) DFT of a contiguous vector (out != in). */
void ora_dft(const cplx* in, cplx* out, int64_t n, int sign) {
    for (int64_t m = 0; m < n; m++) {
        cplx s = 0.0;
        for (int64_t j = 0; j < n; j++) {
            int64_t t = (j * m) % n;
            double ang = sign * 2.0 * ORA_PI * (double)t / (double)n;
            s += in[j] * (cos(ang) + I * sin(ang));
        }
        out[m] = s;
    }
}

/* Iterative radix-2 Cooley-Tukey FFT, in place; n must be a power of two. */
void ora_fft(cplx* x, int64_t n, int sign) {
    /* bit-reversal permutation */
    for (int64_t i = 1, j = 0; i < n; i++) {
        int64_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) {
            cplx t = x[i];
            x[i] = x[j];
            x[j] = t;
        }
    }
    for (int64_t len = 2; len <= n; len <<= 1) {
        int64_t half = len / 2;
        for (int64_t k = 0; k < half; k++) {
            double ang = sign * 2.0 * ORA_PI * (double)k / (double)len;
            cplx w = cos(ang) + I * sin(ang);
            for (int64_t i = 0; i < n; i += len) {
                cplx u = x[i + k];
                cplx v = x[i + k + half] * w;
                x[i + k] = u + v;
                x[i + k + half] = u - v;
            }
        }
    }
}

/* Multi-dimensional transform of one instance: a 1D FFT along every line of every
 * axis (the factorisation over the tensor-product lattice, Sec. 3.2). */
static void fft_nd(const ora_problem* p, cplx* f, int sign) {
    for (int a = 0; a < p->ndim; a++) {
        int64_t n = p->n[a];
        int64_t stride = (a == 0) ? 1 : (a == 1 ? p->n[0] : p->n[0] * p->n[1]);
        int64_t nlines = npts(p) / n;
#pragma omp parallel
        {
            cplx* buf = (cplx*)malloc(sizeof(cplx) * (size_t)n);
#pragma omp for schedule(static)
            for (int64_t line = 0; line < nlines; line++) {
                /* base index of this line: split line into (below, above) the axis */
                int64_t below = line % stride;
                int64_t above = line / stride;
                int64_t base = below + above * stride * n;
                for (int64_t i = 0; i < n; i++) buf[i] = f[base + i * stride];
                ora_fft(buf, n, sign);
                for (int64_t i = 0; i < n; i++) f[base + i * stride] = buf[i];
            }
            free(buf);
        }
    }
}

/* E(k) = exp(L(k) h/2) on the full spectral lattice (reading R2), with the 1/M of the
 * inverse transform folded in. */
static cplx* make_E(const ora_problem* p, double sign_of_phase) {
    int64_t M = npts(p);
    cplx* E = (cplx*)malloc(sizeof(cplx) * (size_t)M);
    for (int64_t j = 0; j < M; j++) {
        int64_t idx[3];
        unflatten(p, j, idx);
        double k2 = 0.0;
        for (int a = 0; a < p->ndim; a++) {
            double k = k_of(p, a, idx[a]);
            k2 += k * k;
        }
        cplx L = -I * sign_of_phase * p->alpha * k2 - p->gamma;
        E[j] = cexp(L * p->h / 2.0) / (double)M;
    }
    return E;
}

/* e^{L h/2} in the cosine or sine basis of a 1D half domain (reading R12): the DCT-II or
 * DST-II sums, the multiply by exp(L(k_m) h/2), and the matching inverse sums (weights
 * 1, 2, ..., 2 for the cosines and 2, ..., 2, 1 for the sines, over n). The angles
 * pi q / (2n) come from one table indexed by q = m'(2j + 1) mod 4n. */
static void apply_D_basis(const ora_problem* p, cplx* f, double sign_of_phase) {
    int64_t n = p->n[0];
    double L = p->hi[0] - p->lo[0];
    int sine = p->basis == 2;
    double* ct = (double*)malloc(sizeof(double) * 4 * (size_t)n);
    double* st = (double*)malloc(sizeof(double) * 4 * (size_t)n);
    for (int64_t q = 0; q < 4 * n; q++) {
        ct[q] = cos(ORA_PI * (double)q / (2.0 * (double)n));
        st[q] = sin(ORA_PI * (double)q / (2.0 * (double)n));
    }
    cplx* c = (cplx*)malloc(sizeof(cplx) * (size_t)n);
#pragma omp parallel for schedule(static)
    for (int64_t m = 0; m < n; m++) {
        int64_t mm = m + sine;
        cplx acc = 0.0;
        for (int64_t j = 0; j < n; j++) {
            int64_t q = (mm * (2 * j + 1)) % (4 * n);
            acc += f[j] * (sine ? st[q] : ct[q]);
        }
        double k = ORA_PI * (double)mm / L;
        c[m] = acc * cexp((-I * sign_of_phase * p->alpha * k * k - p->gamma) * p->h / 2.0);
    }
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; j++) {
        cplx acc = 0.0;
        for (int64_t m = 0; m < n; m++) {
            int64_t mm = m + sine;
            int64_t q = (mm * (2 * j + 1)) % (4 * n);
            double w = sine ? (m == n - 1 ? 1.0 : 2.0) : (m == 0 ? 1.0 : 2.0);
            acc += w * c[m] * (sine ? st[q] : ct[q]);
        }
        f[j] = acc / (double)n;
    }
    free(ct);
    free(st);
    free(c);
}

/* D f = F^{-1}[E F[f]]: the interaction-picture propagator e^{L h/2} applied by a
 * local multiplication in the spectral basis (Sec. 3.6, last paragraph). */
static void apply_D(const ora_problem* p, const cplx* E, cplx* f) {
    if (p->basis) {
        apply_D_basis(p, f, 1.0);
        return;
    }
    int64_t M = npts(p);
    fft_nd(p, f, -1);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < M; j++) f[j] *= E[j];
    fft_nd(p, f, +1);
}

/* ------------------------------------------------------------------------------------
 * Philox4x32-10 (Salmon et al., SC'11): 10 rounds of the Philox S-box with
 * multipliers 0xD2511F53, 0xCD9E8D57 and Weyl key increments 0x9E3779B9, 0xBB67AE85.
 * ---------------------------------------------------------------------------------- */
void ora_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; r++) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* Raw words for a block of counters (test entry): ctr is [count][4]. */
void ora_philox_batch(const uint32_t* ctr, int64_t count, uint64_t seed, uint32_t* out) {
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int64_t i = 0; i < count; i++) ora_philox4x32_10(ctr + 4 * i, key, out + 4 * i);
}

/* Complex standard normal z (E|z|^2 = 2) for point j of an instance at a step and tag
 * (reading R4), Box-Muller on two uniforms made exact in 24 bits. */
static cplx noise_z(uint64_t seed, uint32_t inst, int64_t step, uint32_t tag, int64_t j) {
    uint32_t ctr[4], key[2], r[4];
    uint64_t q = (uint64_t)j >> 1;
    uint64_t st = (uint64_t)step;
    ctr[0] = (uint32_t)q;
    ctr[1] = inst;
    ctr[2] = (uint32_t)st;
    ctr[3] = (tag << 24) | (uint32_t)((st >> 32) & 0xFFFFFFu);
    key[0] = (uint32_t)seed;
    key[1] = (uint32_t)(seed >> 32);
    ora_philox4x32_10(ctr, key, r);
    uint32_t ra = (j & 1) ? r[2] : r[0];
    uint32_t rb = (j & 1) ? r[3] : r[1];
    double u1 = ((double)(ra >> 8) + 1.0) * 0x1.0p-24;
    double u2 = (double)(rb >> 8) * 0x1.0p-24;
    double rad = sqrt(-2.0 * log(u1));
    return rad * (cos(2.0 * ORA_PI * u2) + I * sin(2.0 * ORA_PI * u2));
}

/* The noise of one instance at step `step`: xi[0..M) and, when the potential is noisy
 * (R10), eta in the real parts of xi[M..2M) (test entries and used by G). */
static void noise_field(const ora_problem* p, int64_t b, int64_t step, cplx* xi) {
    int64_t M = npts(p);
    double scale = 1.0 / sqrt(2.0 * p->h * dV_of(p));
    double vscale = 1.0 / sqrt(p->h * dV_of(p));
    uint32_t inst = p->id_base + (uint32_t)b;
    int64_t S = p->noise_substeps > 1 ? (int64_t)p->noise_substeps : 1;
    double inv_sqrt_S = 1.0 / sqrt((double)S);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < M; j++) {
        cplx z = 0.0, zv = 0.0;
        for (int64_t q = 0; q < S; q++) {
            z += noise_z(p->seed, inst, step * S + q, 0u, j);
            if (p->sigma_V != 0.0) zv += noise_z(p->seed, inst, step * S + q, 3u, j);
        }
        xi[j] = scale * inv_sqrt_S * z;
        if (p->sigma_V != 0.0) xi[M + j] = vscale * inv_sqrt_S * creal(zv);
    }
}

/* eta [batch][M] of a step (R10). */
void ora_vnoise(const ora_problem* p, int64_t step, double* eta) {
    int64_t M = npts(p);
    cplx* buf = (cplx*)malloc(sizeof(cplx) * 2 * (size_t)M);
    for (int64_t b = 0; b < p->batch; b++) {
        noise_field(p, b, step, buf);
        for (int64_t j = 0; j < M; j++) eta[b * M + j] = p->sigma_V != 0.0 ? creal(buf[M + j]) : 0.0;
    }
    free(buf);
}

/* Does a step draw noise (additive or in the potential)? */
static int noisy(const ora_problem* p) { return p->sigma != 0.0 || p->sigma_V != 0.0; }

void ora_noise(const ora_problem* p, int64_t step, cplx* xi /* [batch][M] */) {
    int64_t M = npts(p);
    cplx* buf = (cplx*)malloc(sizeof(cplx) * 2 * (size_t)M);
    for (int64_t b = 0; b < p->batch; b++) {
        noise_field(p, b, step, buf);
        memcpy(xi + b * M, buf, sizeof(cplx) * (size_t)M);
    }
    free(buf);
}

/* ------------------------------------------------------------------------------------
 * Right-hand side G (reading R3): -i (V + g|phi|^2) phi + sigma xi.
 * ---------------------------------------------------------------------------------- */

/* Potential of instance b on the lattice: trap part plus the optional grid. */
static void potential(const ora_problem* p, int64_t b, double* V) {
    int64_t M = npts(p);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < M; j++) {
        int64_t idx[3];
        unflatten(p, j, idx);
        double v = 0.0;
        for (int a = 0; a < p->ndim; a++) {
            double x = p->lo[a] + ((double)idx[a] + (p->basis ? 0.5 : 0.0)) * dx_of(p, a);
            v += 0.5 * p->trap[a] * x * x;
        }
        if (p->Vgrid) v += p->Vgrid[b * M + j];
        V[j] = v;
    }
}

/* The non-local potential of one instance (R11): the periodic convolution written out. */
static void conv_potential(const ora_problem* p, const cplx* phi, double* out) {
    int64_t n = p->n[0];
    double dv = dV_of(p);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        double s = 0.0;
        for (int64_t j = 0; j < n; j++) {
            double rho = creal(phi[j]) * creal(phi[j]) + cimag(phi[j]) * cimag(phi[j]);
            s += p->convK[(i - j + n) % n] * rho;
        }
        out[i] = dv * s;
    }
}

static int check_problem(const ora_problem* p);

/* V_c of every instance of psi [batch][n] (test entry; 1D with a kernel). */
int ora_conv_potential(const ora_problem* p, const cplx* psi, double* out) {
    if (check_problem(p) || !p->convK) return -1;
    int64_t M = npts(p);
    for (int64_t b = 0; b < p->batch; b++) conv_potential(p, psi + b * M, out + b * M);
    return 0;
}

/* out = h * G(phi); xi is the step's noise buffer (noise_field) or NULL */
static void hG(const ora_problem* p, const double* V, const cplx* xi, const cplx* phi, cplx* out) {
    int64_t M = npts(p);
    double* vc = NULL;
    if (p->convK) {
        vc = (double*)malloc(sizeof(double) * (size_t)M);
        conv_potential(p, phi, vc);
    }
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < M; j++) {
        double m2 = creal(phi[j]) * creal(phi[j]) + cimag(phi[j]) * cimag(phi[j]);
        double veff = V[j];
        if (vc) veff += vc[j];
        if (xi && p->sigma_V != 0.0) veff += p->sigma_V * creal(xi[M + j]);
        cplx g = -I * (veff + p->gnl * m2) * phi[j];
        if (xi) g += p->sigma * xi[j];
        out[j] = p->h * g;
    }
    free(vc);
}

static void apply_D_dense(const ora_problem* p, const cplx* E, cplx* f);

/* ------------------------------------------------------------------------------------
 * One RK4IP step of one instance (reading R1). Work buffers are allocated per call.
 * With dense != 0 every D goes through dense DFT sums instead of the FFT.
 * ---------------------------------------------------------------------------------- */
#define DAPPLY(f) (dense ? apply_D_dense(p, E, (f)) : apply_D(p, E, (f)))
static void step_one_x(const ora_problem* p, const cplx* E, const double* V, const cplx* xi, cplx* psi, int dense) {
    int64_t M = npts(p);
    size_t bytes = sizeof(cplx) * (size_t)M;
    cplx* a = (cplx*)malloc(bytes);
    cplx* k1 = (cplx*)malloc(bytes);
    cplx* k2 = (cplx*)malloc(bytes);
    cplx* k3 = (cplx*)malloc(bytes);
    cplx* k4 = (cplx*)malloc(bytes);
    cplx* t = (cplx*)malloc(bytes);

    /* a = D psi_n : the state moved to the interaction picture of the midpoint */
    memcpy(a, psi, bytes);
    DAPPLY(a);
    /* k1 = D[h G(psi_n)] : eq. (6) evaluated at t_n */
    hG(p, V, xi, psi, k1);
    DAPPLY(k1);
    /* k2 = h G(a + k1/2) : at the midpoint the picture change is the identity */
    for (int64_t j = 0; j < M; j++) t[j] = a[j] + 0.5 * k1[j];
    hG(p, V, xi, t, k2);
    /* k3 = h G(a + k2/2) */
    for (int64_t j = 0; j < M; j++) t[j] = a[j] + 0.5 * k2[j];
    hG(p, V, xi, t, k3);
    /* k4 = h G(D(a + k3)) : eq. (6) at t_n + h, mapped back through D D^{-1} */
    for (int64_t j = 0; j < M; j++) t[j] = a[j] + k3[j];
    DAPPLY(t);
    hG(p, V, xi, t, k4);
    /* psi_{n+1} = D(a + k1/6 + k2/3 + k3/3) + k4/6 */
    for (int64_t j = 0; j < M; j++) t[j] = a[j] + k1[j] / 6.0 + k2[j] / 3.0 + k3[j] / 3.0;
    DAPPLY(t);
    for (int64_t j = 0; j < M; j++) psi[j] = t[j] + k4[j] / 6.0;

    free(a);
    free(k1);
    free(k2);
    free(k3);
    free(k4);
    free(t);
}

/* One semi-implicit step of one instance in the interaction picture (reading R6). */
static void si_step_one_x(const ora_problem* p, const cplx* E, const double* V, const cplx* xi, cplx* psi,
                          int dense) {
    int64_t M = npts(p);
    size_t bytes = sizeof(cplx) * (size_t)M;
    cplx* a = (cplx*)malloc(bytes);
    cplx* m = (cplx*)malloc(bytes);
    cplx* t = (cplx*)malloc(bytes);
    /* a = D psi_n: the state in the picture of the midpoint */
    memcpy(a, psi, bytes);
    DAPPLY(a);
    /* the midpoint value m = a + (h/2) G(m), by three fixed-point iterations from m = a
     * (at the midpoint the picture change is the identity) */
    memcpy(m, a, bytes);
    for (int it = 0; it < 3; it++) {
        hG(p, V, xi, m, t);
        for (int64_t j = 0; j < M; j++) m[j] = a[j] + 0.5 * t[j];
    }
    /* end of the step in the midpoint picture, 2 m - a, mapped back through D */
    for (int64_t j = 0; j < M; j++) t[j] = 2.0 * m[j] - a[j];
    DAPPLY(t);
    memcpy(psi, t, bytes);
    free(a);
    free(m);
    free(t);
}

#undef DAPPLY

static void step_one(const ora_problem* p, const cplx* E, const double* V, const cplx* xi, cplx* psi) {
    if (p->integrator == 1)
        si_step_one_x(p, E, V, xi, psi, 0);
    else
        step_one_x(p, E, V, xi, psi, 0);
}

static int check_problem(const ora_problem* p) {
    if (p->ndim < 1 || p->ndim > 3) return -1;
    for (int a = 0; a < 3; a++) {
        int64_t n = p->n[a];
        if (a >= p->ndim) {
            if (n != 1) return -1;
            continue;
        }
        if (n < 2 || (n & (n - 1)) != 0) return -1;
        if (!(p->hi[a] > p->lo[a])) return -1;
    }
    if (p->batch < 1 || !(p->h > 0.0)) return -1;
    if (p->integrator != 0 && p->integrator != 1) return -1;
    if (p->noise_substeps > 1 && (p->noise_substeps & (p->noise_substeps - 1)) != 0) return -1;
    if (!isfinite(p->sigma_V)) return -1;
    if (p->convK && p->ndim != 1) return -1;
    if (p->basis < 0 || p->basis > 2 || (p->basis && (p->ndim != 1 || p->convK))) return -1;
    return 0;
}

/* The tangent and the adjoint cover G without the noisy or non-local potential (the
 * adaptive integrator takes the non-local one; it is deterministic, so not the noise). */
static int plain_potential(const ora_problem* p) { return p->sigma_V == 0.0 && p->convK == NULL && !p->basis; }

/* Advance every instance by nsteps steps, the first one having index step0. */
static int run_steps(const ora_problem* p, cplx* psi, int64_t step0, int64_t nsteps) {
    int64_t M = npts(p);
    cplx* E = make_E(p, 1.0);
    double* V = (double*)malloc(sizeof(double) * (size_t)M);
    cplx* xi = noisy(p) ? (cplx*)malloc(sizeof(cplx) * 2 * (size_t)M) : NULL;
    for (int64_t b = 0; b < p->batch; b++) {
        potential(p, b, V);
        for (int64_t s = 0; s < nsteps; s++) {
            if (xi) noise_field(p, b, step0 + s, xi);
            step_one(p, E, V, xi, psi + b * M);
        }
    }
    free(E);
    free(V);
    free(xi);
    return 0;
}

int ora_step(const ora_problem* p, cplx* psi, int64_t step_index) {
    if (check_problem(p)) return -1;
    return run_steps(p, psi, step_index, 1);
}

/* One step of every instance with dense DFT sums in place of the FFT (tiny lattices). */
int ora_step_dense(const ora_problem* p, cplx* psi, int64_t step_index) {
    if (check_problem(p)) return -1;
    int64_t M = npts(p);
    cplx* E = make_E(p, 1.0);
    double* V = (double*)malloc(sizeof(double) * (size_t)M);
    cplx* xi = noisy(p) ? (cplx*)malloc(sizeof(cplx) * 2 * (size_t)M) : NULL;
    for (int64_t b = 0; b < p->batch; b++) {
        potential(p, b, V);
        if (xi) noise_field(p, b, step_index, xi);
        if (p->integrator == 1)
            si_step_one_x(p, E, V, xi, psi + b * M, 1);
        else
            step_one_x(p, E, V, xi, psi + b * M, 1);
    }
    free(E);
    free(V);
    free(xi);
    return 0;
}

/* ------------------------------------------------------------------------------------
 * Integrals of the field (Sec. 2 property 2; quadrature with the uniform weights dV of
 * a Fourier lattice, Sec. 3.4). out[b][4] = {N, E_kin, E_pot, E_int}:
 *   N     = dV sum |psi|^2
 *   E_kin = alpha dV sum_a sum_j |d_a psi_j|^2, d_a psi = F^{-1}[i k_a F psi]
 *   E_pot = dV sum V |psi|^2
 *   E_int = dV sum (g/2) |psi|^4
 * ---------------------------------------------------------------------------------- */
void ora_diag(const ora_problem* p, const cplx* psi, double* out) {
    int64_t M = npts(p);
    double dV = dV_of(p);
    double* V = (double*)malloc(sizeof(double) * (size_t)M);
    cplx* d = (cplx*)malloc(sizeof(cplx) * (size_t)M);
    for (int64_t b = 0; b < p->batch; b++) {
        const cplx* f = psi + b * M;
        potential(p, b, V);
        double N = 0.0, Ep = 0.0, Ei = 0.0, Ek = 0.0;
        for (int64_t j = 0; j < M; j++) {
            double m2 = creal(f[j]) * creal(f[j]) + cimag(f[j]) * cimag(f[j]);
            N += m2;
            Ep += V[j] * m2;
            Ei += 0.5 * p->gnl * m2 * m2;
        }
        for (int a = 0; a < p->ndim; a++) {
            memcpy(d, f, sizeof(cplx) * (size_t)M);
            fft_nd(p, d, -1);
            for (int64_t j = 0; j < M; j++) {
                int64_t idx[3];
                unflatten(p, j, idx);
                d[j] *= I * k_of(p, a, idx[a]) / (double)M;
            }
            fft_nd(p, d, +1);
            for (int64_t j = 0; j < M; j++) Ek += creal(d[j]) * creal(d[j]) + cimag(d[j]) * cimag(d[j]);
        }
        out[4 * b + 0] = dV * N;
        out[4 * b + 1] = p->alpha * dV * Ek;
        out[4 * b + 2] = dV * Ep;
        out[4 * b + 3] = dV * Ei;
    }
    free(V);
    free(d);
}

/* Overlap c_b = dV sum conj(phi_j) psi_bj with one target phi shared by all instances. */
void ora_overlap(const ora_problem* p, const cplx* phi, const cplx* psi, cplx* out) {
    int64_t M = npts(p);
    double dV = dV_of(p);
    for (int64_t b = 0; b < p->batch; b++) {
        cplx c = 0.0;
        for (int64_t j = 0; j < M; j++) c += conj(phi[j]) * psi[b * M + j];
        out[b] = dV * c;
    }
}

/* Moments over paths (Sec. 3.5, many paths): per point, mean of |psi|^2 and its sample
 * variance with the (P-1) divisor. */
void ora_moments(const ora_problem* p, const cplx* psi, double* mean, double* var) {
    int64_t M = npts(p);
    int64_t P = p->batch;
    for (int64_t j = 0; j < M; j++) {
        double s = 0.0;
        for (int64_t b = 0; b < P; b++) {
            cplx v = psi[b * M + j];
            s += creal(v) * creal(v) + cimag(v) * cimag(v);
        }
        double mu = s / (double)P;
        double ss = 0.0;
        for (int64_t b = 0; b < P; b++) {
            cplx v = psi[b * M + j];
            double d = creal(v) * creal(v) + cimag(v) * cimag(v) - mu;
            ss += d * d;
        }
        mean[j] = mu;
        var[j] = P > 1 ? ss / (double)(P - 1) : 0.0;
    }
}

/* Run with samples and checkpoints.
 *   diag: [nsamples][batch][4] with samples at relative steps 0, s, 2s, ... <= nsteps
 *         (nsamples = nsteps/s + 1), or NULL.
 *   ckpt: [ceil(nsteps/M)][batch*Mpts], the state at relative steps 0, M, 2M, ... < nsteps,
 *         or NULL. */
int ora_run(const ora_problem* p, cplx* psi, int64_t step0, int64_t nsteps, int64_t sample_every, double* diag,
            cplx* ckpt, int64_t ckpt_every) {
    if (check_problem(p) || nsteps < 0) return -1;
    if (diag && sample_every < 1) return -1;
    if (ckpt && ckpt_every < 1) return -1;
    int64_t tot = npts(p) * p->batch;
    int64_t sample = 0;
    for (int64_t s = 0; s <= nsteps; s++) {
        if (diag && s % sample_every == 0) {
            ora_diag(p, psi, diag + sample * p->batch * 4);
            sample++;
        }
        if (s == nsteps) break;
        if (ckpt && s % ckpt_every == 0) memcpy(ckpt + (s / ckpt_every) * tot, psi, sizeof(cplx) * (size_t)tot);
        run_steps(p, psi, step0 + s, 1);
    }
    return 0;
}

/* ------------------------------------------------------------------------------------
 * Tangent-linear model and discrete adjoint of the step above (not in the paper).
 * The step is R-linear in (psi, conj psi); with the real inner product
 * <x,y> = Re sum conj(x) y the transposes are
 *   D^T = F^{-1} conj(E) F,
 *   (dG)^T lam = conj(A) lam + B conj(lam),  A = -i(V + 2g|phi|^2),  B = -i g phi^2,
 *   dG/dV contribution:  Vbar_j += Im(conj(lam_j) phi_j).
 * Gradients follow the convention d/dRe + i d/dIm.
 * ---------------------------------------------------------------------------------- */

/* out = h * dG(phi)[dphi] - i h dV phi */
static void hdG(const ora_problem* p, const double* V, const double* dV, const cplx* phi, const cplx* dphi,
                cplx* out) {
    int64_t M = npts(p);
    for (int64_t j = 0; j < M; j++) {
        double m2 = creal(phi[j]) * creal(phi[j]) + cimag(phi[j]) * cimag(phi[j]);
        cplx A = -I * (V[j] + 2.0 * p->gnl * m2);
        cplx B = -I * p->gnl * phi[j] * phi[j];
        cplx g = A * dphi[j] + B * conj(dphi[j]);
        if (dV) g += -I * dV[j] * phi[j];
        out[j] = p->h * g;
    }
}

/* lam_out = h (dG(phi))^T lam_in; Vbar += h Im(conj(lam_in) phi) */
static void hdG_T(const ora_problem* p, const double* V, const cplx* phi, const cplx* lam, cplx* out, double* Vbar) {
    int64_t M = npts(p);
    for (int64_t j = 0; j < M; j++) {
        double m2 = creal(phi[j]) * creal(phi[j]) + cimag(phi[j]) * cimag(phi[j]);
        cplx A = -I * (V[j] + 2.0 * p->gnl * m2);
        cplx B = -I * p->gnl * phi[j] * phi[j];
        out[j] = p->h * (conj(A) * lam[j] + B * conj(lam[j]));
        if (Vbar) Vbar[j] += p->h * cimag(conj(lam[j]) * phi[j]);
    }
}

/* Tangent step of one instance: (psi, dpsi) -> (psi', dpsi') for a perturbation dV of
 * the potential grid (dV may be NULL). */
static void tangent_one(const ora_problem* p, const cplx* E, const double* V, const double* dVg, const cplx* xi,
                        cplx* psi, cplx* dpsi) {
    int64_t M = npts(p);
    size_t bytes = sizeof(cplx) * (size_t)M;
    cplx *a = malloc(bytes), *k1 = malloc(bytes), *k2 = malloc(bytes), *k3 = malloc(bytes), *k4 = malloc(bytes);
    cplx *da = malloc(bytes), *dk1 = malloc(bytes), *dk2 = malloc(bytes), *dk3 = malloc(bytes), *dk4 = malloc(bytes);
    cplx *t = malloc(bytes), *dt = malloc(bytes);

    memcpy(a, psi, bytes);
    apply_D(p, E, a);
    memcpy(da, dpsi, bytes);
    apply_D(p, E, da);
    hG(p, V, xi, psi, k1);
    hdG(p, V, dVg, psi, dpsi, dk1);
    apply_D(p, E, k1);
    apply_D(p, E, dk1);
    for (int64_t j = 0; j < M; j++) {
        t[j] = a[j] + 0.5 * k1[j];
        dt[j] = da[j] + 0.5 * dk1[j];
    }
    hG(p, V, xi, t, k2);
    hdG(p, V, dVg, t, dt, dk2);
    for (int64_t j = 0; j < M; j++) {
        t[j] = a[j] + 0.5 * k2[j];
        dt[j] = da[j] + 0.5 * dk2[j];
    }
    hG(p, V, xi, t, k3);
    hdG(p, V, dVg, t, dt, dk3);
    for (int64_t j = 0; j < M; j++) {
        t[j] = a[j] + k3[j];
        dt[j] = da[j] + dk3[j];
    }
    apply_D(p, E, t);
    apply_D(p, E, dt);
    hG(p, V, xi, t, k4);
    hdG(p, V, dVg, t, dt, dk4);
    for (int64_t j = 0; j < M; j++) {
        t[j] = a[j] + k1[j] / 6.0 + k2[j] / 3.0 + k3[j] / 3.0;
        dt[j] = da[j] + dk1[j] / 6.0 + dk2[j] / 3.0 + dk3[j] / 3.0;
    }
    apply_D(p, E, t);
    apply_D(p, E, dt);
    for (int64_t j = 0; j < M; j++) {
        psi[j] = t[j] + k4[j] / 6.0;
        dpsi[j] = dt[j] + dk4[j] / 6.0;
    }
    free(a); free(k1); free(k2); free(k3); free(k4);
    free(da); free(dk1); free(dk2); free(dk3); free(dk4);
    free(t); free(dt);
}

/* Tangent-linear run: advances psi and dpsi by nsteps; dV is [batch][M] or NULL. */
int ora_tangent(const ora_problem* p, cplx* psi, cplx* dpsi, const double* dV, int64_t step0, int64_t nsteps) {
    /* the RK4IP step's tangent only, with the plain potential */
    if (check_problem(p) || p->integrator != 0 || !plain_potential(p)) return -1;
    int64_t M = npts(p);
    cplx* E = make_E(p, 1.0);
    double* V = malloc(sizeof(double) * (size_t)M);
    cplx* xi = p->sigma != 0.0 ? malloc(sizeof(cplx) * (size_t)M) : NULL;
    for (int64_t b = 0; b < p->batch; b++) {
        potential(p, b, V);
        for (int64_t s = 0; s < nsteps; s++) {
            if (xi) noise_field(p, b, step0 + s, xi);
            tangent_one(p, E, V, dV ? dV + b * M : NULL, xi, psi + b * M, dpsi + b * M);
        }
    }
    free(E);
    free(V);
    free(xi);
    return 0;
}

/* Adjoint of one step of one instance: given psi_n and lam = adjoint of psi_{n+1},
 * overwrite lam with the adjoint of psi_n and add this step's share to Vbar. */
static void adjoint_one(const ora_problem* p, const cplx* E, const cplx* Ec, const double* V, const cplx* xi,
                        const cplx* psi, cplx* lam, double* Vbar) {
    int64_t M = npts(p);
    size_t bytes = sizeof(cplx) * (size_t)M;
    cplx *a = malloc(bytes), *k1 = malloc(bytes), *k2 = malloc(bytes), *k3 = malloc(bytes);
    cplx *p2 = malloc(bytes), *p3 = malloc(bytes), *w = malloc(bytes);
    cplx *abar = malloc(bytes), *k1bar = malloc(bytes), *k2bar = malloc(bytes), *k3bar = malloc(bytes);
    cplx *accbar = malloc(bytes), *wbar = malloc(bytes), *tmp = malloc(bytes), *g0bar = malloc(bytes);

    /* forward recomputation of the stage inputs */
    memcpy(a, psi, bytes);
    apply_D(p, E, a);
    hG(p, V, xi, psi, k1);
    apply_D(p, E, k1);
    for (int64_t j = 0; j < M; j++) p2[j] = a[j] + 0.5 * k1[j];
    hG(p, V, xi, p2, k2);
    for (int64_t j = 0; j < M; j++) p3[j] = a[j] + 0.5 * k2[j];
    hG(p, V, xi, p3, k3);
    for (int64_t j = 0; j < M; j++) w[j] = a[j] + k3[j];
    apply_D(p, E, w);

    /* psi' = D acc + k4/6  ->  accbar = D^T lam, k4bar = lam/6 */
    memcpy(accbar, lam, bytes);
    apply_D(p, Ec, accbar);
    for (int64_t j = 0; j < M; j++) tmp[j] = lam[j] / 6.0;
    /* k4 = h G(w) -> wbar = h dG(w)^T k4bar */
    hdG_T(p, V, w, tmp, wbar, Vbar);
    /* w = D u -> ubar = D^T wbar (kept in wbar) */
    apply_D(p, Ec, wbar);
    /* acc = a + k1/6 + k2/3 + k3/3 ; u = a + k3 */
    for (int64_t j = 0; j < M; j++) {
        abar[j] = accbar[j] + wbar[j];
        k1bar[j] = accbar[j] / 6.0;
        k2bar[j] = accbar[j] / 3.0;
        k3bar[j] = accbar[j] / 3.0 + wbar[j];
    }
    /* k3 = h G(p3), p3 = a + k2/2 */
    hdG_T(p, V, p3, k3bar, tmp, Vbar);
    for (int64_t j = 0; j < M; j++) {
        abar[j] += tmp[j];
        k2bar[j] += 0.5 * tmp[j];
    }
    /* k2 = h G(p2), p2 = a + k1/2 */
    hdG_T(p, V, p2, k2bar, tmp, Vbar);
    for (int64_t j = 0; j < M; j++) {
        abar[j] += tmp[j];
        k1bar[j] += 0.5 * tmp[j];
    }
    /* k1 = D g0 -> g0bar = D^T k1bar; g0 = h G(psi) */
    memcpy(g0bar, k1bar, bytes);
    apply_D(p, Ec, g0bar);
    hdG_T(p, V, psi, g0bar, tmp, Vbar);
    /* a = D psi -> psibar = D^T abar + (from g0) */
    apply_D(p, Ec, abar);
    for (int64_t j = 0; j < M; j++) lam[j] = abar[j] + tmp[j];

    free(a); free(k1); free(k2); free(k3); free(p2); free(p3); free(w);
    free(abar); free(k1bar); free(k2bar); free(k3bar); free(accbar); free(wbar); free(tmp); free(g0bar);
}

/* Gradient of a loss with adjoint lamT at psi after nsteps (started at step0) with
 * respect to psi0 and to the potential grid. Checkpoints every ckpt_every steps; each
 * segment is recomputed from its checkpoint and walked backwards.
 *   grad_psi0: [batch][M] (out);  grad_V: [batch][M] (out) or NULL. */
int ora_adjoint(const ora_problem* p, const cplx* psi0, int64_t step0, int64_t nsteps, int64_t ckpt_every,
                const cplx* lamT, cplx* grad_psi0, double* grad_V) {
    /* the discrete adjoint of the RK4IP step only, with the plain potential */
    if (check_problem(p) || p->integrator != 0 || !plain_potential(p) || nsteps < 0 || ckpt_every < 1) return -1;
    int64_t M = npts(p);
    size_t bytes = sizeof(cplx) * (size_t)M;
    cplx* E = make_E(p, 1.0);
    cplx* Ec = make_E(p, -1.0); /* conj(E): same damping, opposite phase */
    double* V = malloc(sizeof(double) * (size_t)M);
    cplx* xi = p->sigma != 0.0 ? malloc(bytes) : NULL;
    int64_t nseg = (nsteps + ckpt_every - 1) / ckpt_every;
    cplx* ck = malloc(bytes * (size_t)(nseg > 0 ? nseg : 1));
    cplx* states = malloc(bytes * (size_t)ckpt_every);
    for (int64_t b = 0; b < p->batch; b++) {
        potential(p, b, V);
        double* Vbar = grad_V ? grad_V + b * M : NULL;
        if (Vbar) memset(Vbar, 0, sizeof(double) * (size_t)M);
        /* forward sweep storing one state per segment start */
        cplx* f = malloc(bytes);
        memcpy(f, psi0 + b * M, bytes);
        for (int64_t s = 0; s < nsteps; s++) {
            if (s % ckpt_every == 0) memcpy(ck + (s / ckpt_every) * M, f, bytes);
            if (xi) noise_field(p, b, step0 + s, xi);
            step_one(p, E, V, xi, f);
        }
        cplx* lam = grad_psi0 + b * M;
        memcpy(lam, lamT + b * M, bytes);
        for (int64_t seg = nseg - 1; seg >= 0; seg--) {
            int64_t s0 = seg * ckpt_every;
            int64_t len = (s0 + ckpt_every <= nsteps) ? ckpt_every : nsteps - s0;
            memcpy(f, ck + seg * M, bytes);
            for (int64_t i = 0; i < len; i++) {
                memcpy(states + i * M, f, bytes);
                if (i + 1 < len) {
                    if (xi) noise_field(p, b, step0 + s0 + i, xi);
                    step_one(p, E, V, xi, f);
                }
            }
            for (int64_t i = len - 1; i >= 0; i--) {
                if (xi) noise_field(p, b, step0 + s0 + i, xi);
                adjoint_one(p, E, Ec, V, xi, states + i * M, lam, Vbar);
            }
        }
        free(f);
    }
    free(E);
    free(Ec);
    free(V);
    free(xi);
    free(ck);
    free(states);
    return 0;
}

/* ------------------------------------------------------------------------------------
 * Brute-force variant for tiny lattices: the same step with D applied through dense
 * DFT matrices (O(M^2)) instead of the FFT. Used only to pin the FFT-based step.
 * ---------------------------------------------------------------------------------- */
/* ------------------------------------------------------------------------------------
 * Adaptive Cash-Karp RK4(5) in the interaction picture (readings R8, R9).
 * ---------------------------------------------------------------------------------- */

/* The Cash-Karp embedded pair: nodes c, stage matrix a (lower triangle), fifth-order
 * weights b and fourth-order weights b*. */
static const double CK_C[6] = {0.0, 1.0 / 5.0, 3.0 / 10.0, 3.0 / 5.0, 1.0, 7.0 / 8.0};
static const double CK_A[6][5] = {
    {0.0, 0.0, 0.0, 0.0, 0.0},
    {1.0 / 5.0, 0.0, 0.0, 0.0, 0.0},
    {3.0 / 40.0, 9.0 / 40.0, 0.0, 0.0, 0.0},
    {3.0 / 10.0, -9.0 / 10.0, 6.0 / 5.0, 0.0, 0.0},
    {-11.0 / 54.0, 5.0 / 2.0, -70.0 / 27.0, 35.0 / 27.0, 0.0},
    {1631.0 / 55296.0, 175.0 / 512.0, 575.0 / 13824.0, 44275.0 / 110592.0, 253.0 / 4096.0},
};
static const double CK_B5[6] = {37.0 / 378.0, 0.0, 250.0 / 621.0, 125.0 / 594.0, 0.0, 512.0 / 1771.0};
static const double CK_B4[6] = {2825.0 / 27648.0, 0.0, 18575.0 / 48384.0, 13525.0 / 55296.0, 277.0 / 14336.0,
                                1.0 / 4.0};

/* c (6), a (6 x 5, row-major), b (6), b* (6): 48 doubles. */
void ora_ck_tableau(double* out) {
    for (int i = 0; i < 6; i++) out[i] = CK_C[i];
    for (int i = 0; i < 6; i++)
        for (int j = 0; j < 5; j++) out[6 + 5 * i + j] = CK_A[i][j];
    for (int i = 0; i < 6; i++) out[36 + i] = CK_B5[i];
    for (int i = 0; i < 6; i++) out[42 + i] = CK_B4[i];
}

/* f <- e^{L tau} f for one instance (tau of either sign): transform, multiply every mode
 * by exp(L(k) tau) / M, transform back (Sec. 3.6). */
static void apply_exp_L(const ora_problem* p, double tau, cplx* f) {
    int64_t M = npts(p);
    fft_nd(p, f, -1);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < M; j++) {
        int64_t idx[3];
        unflatten(p, j, idx);
        double k2 = 0.0;
        for (int a = 0; a < p->ndim; a++) {
            double k = k_of(p, a, idx[a]);
            k2 += k * k;
        }
        f[j] *= cexp((-I * p->alpha * k2 - p->gamma) * tau) / (double)M;
    }
    fft_nd(p, f, +1);
}

/* One Cash-Karp step of size h of one instance from psi (x space at t_n, which is also the
 * picture frame since the origin is t_n). Writes the fifth-order result at t_n + h (x
 * space) to out and returns the error estimate (reading R8). */
/* out = L f for one instance: transform, multiply every mode by L(k) / M, transform back. */
static void apply_L(const ora_problem* p, const cplx* f, cplx* out) {
    int64_t M = npts(p);
    memcpy(out, f, sizeof(cplx) * (size_t)M);
    fft_nd(p, out, -1);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < M; j++) {
        int64_t idx[3];
        unflatten(p, j, idx);
        double k2 = 0.0;
        for (int a = 0; a < p->ndim; a++) {
            double k = k_of(p, a, idx[a]);
            k2 += k * k;
        }
        out[j] *= (-I * p->alpha * k2 - p->gamma) / (double)M;
    }
    fft_nd(p, out, +1);
}

static double ck_step_one(const ora_problem* p, const double* V, const cplx* psi, double h, cplx* out, int ip) {
    int64_t M = npts(p);
    cplx* k[6];
    for (int i = 0; i < 6; i++) k[i] = (cplx*)malloc(sizeof(cplx) * (size_t)M);
    cplx* y = (cplx*)malloc(sizeof(cplx) * (size_t)M);
    double* vc = p->convK ? (double*)malloc(sizeof(double) * (size_t)M) : NULL;
    for (int i = 0; i < 6; i++) {
        /* stage input in the picture frame, then moved to the stage time */
        for (int64_t j = 0; j < M; j++) {
            cplx v = psi[j];
            for (int q = 0; q < i; q++) v += CK_A[i][q] * k[q][j];
            y[j] = v;
        }
        if (ip && CK_C[i] != 0.0) apply_exp_L(p, CK_C[i] * h, y);
        /* h G at the stage time (G without noise: the method is deterministic only; with
         * the non-local potential of the stage field when there is a kernel, R11) */
        if (vc) conv_potential(p, y, vc);
        for (int64_t j = 0; j < M; j++) {
            double m2 = creal(y[j]) * creal(y[j]) + cimag(y[j]) * cimag(y[j]);
            double veff = vc ? V[j] + vc[j] : V[j];
            k[i][j] = h * (-I * (veff + p->gnl * m2) * y[j]);
        }
        if (ip) {
            /* back to the picture frame */
            if (CK_C[i] != 0.0) apply_exp_L(p, -CK_C[i] * h, k[i]);
        } else {
            /* the explicit method: the linear part in the stage too */
            apply_L(p, y, out);
            for (int64_t j = 0; j < M; j++) k[i][j] += h * out[j];
        }
    }
    double num = 0.0, den = 0.0;
    for (int64_t j = 0; j < M; j++) {
        cplx y5 = psi[j], dlt = 0.0;
        for (int i = 0; i < 6; i++) {
            y5 += CK_B5[i] * k[i][j];
            dlt += (CK_B5[i] - CK_B4[i]) * k[i][j];
        }
        out[j] = y5;
        num += creal(dlt) * creal(dlt) + cimag(dlt) * cimag(dlt);
        den += creal(y5) * creal(y5) + cimag(y5) * cimag(y5);
    }
    if (ip) apply_exp_L(p, h, out);
    for (int i = 0; i < 6; i++) free(k[i]);
    free(y);
    free(vc);
    return sqrt(num / den);
}

static int check_ark45(const ora_problem* p) {
    if (check_problem(p) || p->sigma_V != 0.0 || p->basis) return -1;
    if (p->sigma != 0.0) return -1; /* deterministic only */
    return 0;
}

/* One Cash-Karp step of size h of every instance: out[batch][M] (fifth order, x space),
 * err[batch]. */
int ora_ck_step(const ora_problem* p, const cplx* psi, double h, cplx* out, double* err, int ip) {
    if (check_ark45(p) || !(h > 0.0)) return -1;
    int64_t M = npts(p);
    double* V = (double*)malloc(sizeof(double) * (size_t)M);
    for (int64_t b = 0; b < p->batch; b++) {
        potential(p, b, V);
        err[b] = ck_step_one(p, V, psi + b * M, h, out + b * M, ip);
    }
    free(V);
    return 0;
}

/* The step factor of reading R9. */
static double ck_factor(double err, double tol) {
    if (!isfinite(err)) return 0.2;
    if (err == 0.0) return 5.0;
    double f = 0.9 * pow(tol / err, 0.2);
    return f < 0.2 ? 0.2 : (f > 5.0 ? 5.0 : f);
}

/* Integrate every instance over [0, t_span] with its own adaptive step (readings R8, R9).
 * h[batch]: in, the first trial step; out, the next trial step. stats[batch][2]: accepted
 * and rejected steps. h_log[batch][log_cap] (optional): the accepted step sizes in order.
 * At most max_attempts trial steps per instance. Returns 0 when every instance reached
 * t_span, 1 when one ran out of attempts, -1 on a bad argument. */
int ora_ark45(const ora_problem* p, cplx* psi, double t_span, double tol, int64_t max_attempts, double* h,
              int64_t* stats, double* h_log, int64_t log_cap, int ip) {
    if (check_ark45(p) || !(t_span >= 0.0) || !(tol > 0.0) || max_attempts < 1) return -1;
    int64_t M = npts(p);
    double* V = (double*)malloc(sizeof(double) * (size_t)M);
    cplx* out = (cplx*)malloc(sizeof(cplx) * (size_t)M);
    int rc = 0;
    for (int64_t b = 0; b < p->batch; b++) {
        if (!(h[b] > 0.0)) {
            rc = -1;
            break;
        }
        potential(p, b, V);
        cplx* f = psi + b * M;
        double t = 0.0, hb = h[b];
        int64_t acc = 0, rej = 0;
        while (t < t_span && acc + rej < max_attempts) {
            int last = t + hb >= t_span;
            double htry = last ? t_span - t : hb;
            double err = ck_step_one(p, V, f, htry, out, ip);
            if (err <= tol) {
                memcpy(f, out, sizeof(cplx) * (size_t)M);
                if (h_log && acc < log_cap) h_log[b * log_cap + acc] = htry;
                t = last ? t_span : t + htry;
                acc++;
            } else {
                rej++;
            }
            hb = htry * ck_factor(err, tol);
        }
        if (t < t_span) rc = 1;
        h[b] = hb;
        stats[2 * b] = acc;
        stats[2 * b + 1] = rej;
    }
    free(V);
    free(out);
    return rc;
}

static void apply_D_dense(const ora_problem* p, const cplx* E, cplx* f) {
    if (p->basis) {
        apply_D_basis(p, f, 1.0);  /* already a dense sum */
        return;
    }
    int64_t M = npts(p);
    cplx* F = malloc(sizeof(cplx) * (size_t)M);
    /* forward multi-D DFT by direct summation over all lattice points */
    for (int64_t m = 0; m < M; m++) {
        int64_t im[3];
        unflatten(p, m, im);
        cplx s = 0.0;
        for (int64_t j = 0; j < M; j++) {
            int64_t ij[3];
            unflatten(p, j, ij);
            double ph = 0.0;
            for (int a = 0; a < p->ndim; a++) ph += (double)((ij[a] * im[a]) % p->n[a]) / (double)p->n[a];
            s += f[j] * cexp(-2.0 * ORA_PI * I * ph);
        }
        F[m] = s * E[m];
    }
    for (int64_t j = 0; j < M; j++) {
        int64_t ij[3];
        unflatten(p, j, ij);
        cplx s = 0.0;
        for (int64_t m = 0; m < M; m++) {
            int64_t im[3];
            unflatten(p, m, im);
            double ph = 0.0;
            for (int a = 0; a < p->ndim; a++) ph += (double)((ij[a] * im[a]) % p->n[a]) / (double)p->n[a];
            s += F[m] * cexp(2.0 * ORA_PI * I * ph);
        }
        f[j] = s;
    }
    free(F);
}

int ora_apply_D(const ora_problem* p, cplx* f, int dense, int adjoint) {
    if (check_problem(p)) return -1;
    cplx* E = make_E(p, adjoint ? -1.0 : 1.0);
    int64_t M = npts(p);
    for (int64_t b = 0; b < p->batch; b++) {
        if (p->basis)
            apply_D_basis(p, f + b * M, adjoint ? -1.0 : 1.0);  /* the basis sums are dense */
        else if (dense)
            apply_D_dense(p, E, f + b * M);
        else
            apply_D(p, E, f + b * M);
    }
    free(E);
    return 0;
}

/* Threads the OpenMP loops of the oracle use. */
int ora_threads(void) { return omp_get_max_threads(); }

/* Multi-dimensional unnormalised transform of every instance (test entry). */
int ora_fft_nd(const ora_problem* p, cplx* f, int sign) {
    if (check_problem(p)) return -1;
    int64_t M = npts(p);
    for (int64_t b = 0; b < p->batch; b++) fft_nd(p, f + b * M, sign);
    return 0;
}
