// kernels_ark45.hip -- adaptive Cash-Karp RK4(5) in the interaction picture for 1D
// groups (Sec. 3.5's adaptive fourth-fifth order Runge-Kutta, deterministic only, on
// eq. (6) of Sec. 3.6).
//
// With the picture origin at the start of each step, stage i at t_n + c_i h is
//   Y_i = psi_n + sum_j a_ij k_j,   k_i = e^{-L c_i h} h G(e^{L c_i h} Y_i),
// the step keeps the fifth-order result psi_{n+1} = e^{L h}(psi_n + sum_i b_i k_i), and
// its error estimate is ||sum_i (b_i - b*_i) k_i|| / ||psi_n + sum_i b_i k_i|| (relative
// L2 over the instance). A step is accepted when the estimate is at most tol; either way
// the next trial step is h min(5, max(1/5, 0.9 (tol/err)^{1/5})), and a trial step that
// would pass the end of the interval is cut to end on it.
//
// One workgroup integrates LPB whole lines, each with its own step. A line's state is kept
// in k-space for the whole interval, P = F psi (unnormalised), and so are its stages,
// K_i = F k_i: e^{L tau} is diagonal there, so moving a stage input to its stage time and
// the stage back to the picture frame are per-mode multiplies, and a stage costs one
// transform pair (to evaluate G in x-space) instead of three. Stage I:
//   u = F^{-1}[e^{L c_I h} (P + sum_j a_Ij K_j)] / n,   K_I = e^{-L c_I h} F[h G(u)];
// the step keeps P' = e^{L h}(P + sum_i b_i K_i), and Parseval gives the relative error
// estimate from the k-space sums (the 1/n of both norms cancels). The line is transformed
// once at the start of the launch and back at the end. P, the five stored stages and the
// stage input stay in registers; LDS carries only the FFT exchanges and the error-norm
// partials. e^{L tau} changes with every trial step, so it is formed per mode (phase in
// FP64, reduced to [-pi, pi] before an FP32 sincos) instead of being read from a table.
// Each wave keeps looping while any line of its workgroup is unfinished (the barriers
// are workgroup-wide); a finished line's threads compute and discard. Every line stops
// after max_attempts trial steps, so every wave reaches the end.
#include "pass_common.h"

namespace rk4ip {

namespace {

// The Cash-Karp pair (Cash and Karp, ACM TOMS 16, 201, 1990).
constexpr double kC[6] = {0.0, 1.0 / 5.0, 3.0 / 10.0, 3.0 / 5.0, 1.0, 7.0 / 8.0};
constexpr float kA[6][5] = {
    {0.f, 0.f, 0.f, 0.f, 0.f},
    {(float)(1.0 / 5.0), 0.f, 0.f, 0.f, 0.f},
    {(float)(3.0 / 40.0), (float)(9.0 / 40.0), 0.f, 0.f, 0.f},
    {(float)(3.0 / 10.0), (float)(-9.0 / 10.0), (float)(6.0 / 5.0), 0.f, 0.f},
    {(float)(-11.0 / 54.0), (float)(5.0 / 2.0), (float)(-70.0 / 27.0), (float)(35.0 / 27.0), 0.f},
    {(float)(1631.0 / 55296.0), (float)(175.0 / 512.0), (float)(575.0 / 13824.0), (float)(44275.0 / 110592.0),
     (float)(253.0 / 4096.0)},
};
constexpr double kB5[6] = {37.0 / 378.0, 0.0, 250.0 / 621.0, 125.0 / 594.0, 0.0, 512.0 / 1771.0};
constexpr double kB4[6] = {2825.0 / 27648.0, 0.0, 18575.0 / 48384.0, 13525.0 / 55296.0, 277.0 / 14336.0, 1.0 / 4.0};

constexpr double kHalfPiD = 1.57079632679489661923;
constexpr double kTwoOverPiD = 0.63661977236758134308;

}  // namespace

// sin and cos of an FP64 angle: reduced modulo pi/2 in FP64 to r in [-pi/4, pi/4] and a
// quadrant, then the Taylor series of sin and cos in FP32, cut after the r^11 and r^12
// terms (the first dropped terms are below 1e-11 on that interval, far under FP32's
// rounding). Needs no large-argument reduction, which keeps it short and its registers few.
__device__ __forceinline__ void sincos_fp64_arg(double th, float& sn, float& cs) {
    const double q = rint(th * kTwoOverPiD);
    const float r = (float)fma(-q, kHalfPiD, th);
    const float r2 = r * r;
    float ps = fmaf(r2, -1.0f / 39916800.0f, 1.0f / 362880.0f);
    ps = fmaf(r2, ps, -1.0f / 5040.0f);
    ps = fmaf(r2, ps, 1.0f / 120.0f);
    ps = fmaf(r2, ps, -1.0f / 6.0f);
    const float s0 = fmaf(r * r2, ps, r);
    float pc = fmaf(r2, 1.0f / 479001600.0f, -1.0f / 3628800.0f);
    pc = fmaf(r2, pc, 1.0f / 40320.0f);
    pc = fmaf(r2, pc, -1.0f / 720.0f);
    pc = fmaf(r2, pc, 1.0f / 24.0f);
    pc = fmaf(r2, pc, -0.5f);
    const float c0 = fmaf(r2, pc, 1.0f);
    const int k = (int)((int64_t)q & 3);
    const float a = (k & 1) ? c0 : s0, b = (k & 1) ? s0 : c0;
    sn = (k & 2) ? -a : a;                 // sin(r + k pi/2)
    cs = ((k + 1) & 2) ? -b : b;           // cos(r + k pi/2)
}

// cos and sin of theta = alpha k_m^2 tau for this thread's R modes (the phase of
// e^{L tau} = e^{-gamma tau} e^{-i theta}).
template <class F>
__device__ __forceinline__ void phases(c32 (&cs)[F::R], int t, const ArkArgs& x, double tau) {
    constexpr int R = F::R, T = F::T, N = F::NN;
    const double ph0 = x.alpha * x.kscale * x.kscale * tau;
#pragma unroll
    for (int m = 0; m < R; m++) {
        const int e = t + m * T;
        const double km = (double)(e < N / 2 ? e : e - N);
        float sn, c;
        sincos_fp64_arg(ph0 * km * km, sn, c);
        cs[m] = make_float2(c, sn);
    }
}

// h G(phi) without noise: -i h (V + g |phi|^2) phi
__device__ __forceinline__ c32 hG_ark(const GroupDev& g, c32 phi, float V, float h) {
    const float m2 = fmaf(phi.x, phi.x, phi.y * phi.y);
    const float w = h * fmaf(g.gnl, m2, V);
    return make_float2(w * phi.y, -w * phi.x);
}

// The potential at this thread's R points of line `line` (the trap, plus the grid when
// there is one), formed where G needs it instead of being held in registers.
template <class F>
__device__ __forceinline__ float pot_ark(const GroupDev& g, int t, int m, int64_t line) {
    const int e = t + m * F::T;
    float v = trap_V(g, e, 0, 0);
    if (g.Vgrid) v += g.Vgrid[line * F::NN + e];
    return v;
}

// d <- F[h G(F^{-1} d)] on this thread's R modes of its line (d arrives already scaled by
// 1/n), with the non-local potential of the stage field when CONV.
template <class F, class L, bool CONV>
__device__ __forceinline__ void g_of(c32 (&d)[1][F::R], const GroupDev& g, int64_t line, int t, int l, c32* lds,
                                     const c32* tw, float hf) {
    constexpr int R = F::R;
    fft_line<F, +1, L, 1>(d, t, l, lds, tw);
    if constexpr (CONV) {
        float vc[R];
        conv_V<F, L>(d[0], vc, t, l, lds, tw, g.convK);
#pragma unroll
        for (int m = 0; m < R; m++) d[0][m] = hG_ark(g, d[0][m], pot_ark<F>(g, t, m, line) + vc[m], hf);
    } else {
#pragma unroll
        for (int m = 0; m < R; m++) d[0][m] = hG_ark(g, d[0][m], pot_ark<F>(g, t, m, line), hf);
    }
    fft_line<F, -1, L, 1>(d, t, l, lds, tw);
}

// Stage I (0..5) of a trial step of size h, in k-space: d holds the stage input Y_I and
// leaves as K_I = e^{-L c_I h} F[h G(F^{-1}(e^{L c_I h} Y_I) / n)].
// EX: the explicit comparison method: no picture, K_I = F[h G(F^{-1} Y_I / n)] + h L Y_I.
template <int I, bool CONV, bool EX, class F, class L>
__device__ __forceinline__ void ck_stage(c32 (&d)[1][F::R], const GroupDev& g, int64_t line, int t, int l,
                                         c32* lds, const c32* tw, const ArkArgs& x, double h, float hf) {
    constexpr int R = F::R, T = F::T, N = F::NN;
    constexpr float inv_n = 1.0f / (float)N;  // exact power of two
    if constexpr (EX) {
        // h L(k_m) = -gamma h - i alpha k_m^2 h, applied to Y_I after G's transforms
        c32 y[R];
#pragma unroll
        for (int m = 0; m < R; m++) {
            y[m] = d[0][m];
            d[0][m] = make_float2(d[0][m].x * inv_n, d[0][m].y * inv_n);
        }
        g_of<F, L, CONV>(d, g, line, t, l, lds, tw, hf);
        const double c0 = x.alpha * x.kscale * x.kscale * h;
        const float re = (float)(-x.gamma * h);
#pragma unroll
        for (int m = 0; m < R; m++) {
            const int e = t + m * T;
            const double km = (double)(e < N / 2 ? e : e - N);
            d[0][m] = cadd(d[0][m], cmul(y[m], make_float2(re, (float)(-c0 * km * km))));
        }
    } else if constexpr (I == 0) {
        // c_1 = 0: the stage input is P itself
#pragma unroll
        for (int m = 0; m < R; m++) d[0][m] = make_float2(d[0][m].x * inv_n, d[0][m].y * inv_n);
        g_of<F, L, CONV>(d, g, line, t, l, lds, tw, hf);
    } else {
        const double tau = kC[I] * h;
        c32 cs[R];
        phases<F>(cs, t, x, tau);
        float damp = 1.0f, undamp = 1.0f;  // e^{-gamma tau} and its inverse
        if (x.gamma != 0.0) {
            damp = (float)exp(-x.gamma * tau);
            undamp = (float)exp(x.gamma * tau);
        }
        const float fw = damp * inv_n;
#pragma unroll
        for (int m = 0; m < R; m++) d[0][m] = cmul(d[0][m], make_float2(fw * cs[m].x, -fw * cs[m].y));
        g_of<F, L, CONV>(d, g, line, t, l, lds, tw, hf);
#pragma unroll
        for (int m = 0; m < R; m++) d[0][m] = cmul(d[0][m], make_float2(undamp * cs[m].x, undamp * cs[m].y));
    }
}

// v + a k, componentwise
__device__ __forceinline__ c32 axpy(c32 v, float a, c32 k) { return make_float2(fmaf(a, k.x, v.x), fmaf(a, k.y, v.y)); }

// CONV: G includes the non-local potential (the variant compiled for groups with a kernel).
// EX: the explicit comparison method instead of the interaction picture.
template <int N, int LPB, bool CONV, bool EX>
__global__ void __launch_bounds__((FFTShape<N, 8>::T * LPB)) __attribute__((amdgpu_waves_per_eu(2)))
    k_line_ark45(GroupDev g, float2* __restrict__ psi, ArkArgs x) {
    using F = FFTShape<N, 8>;
    using L = LdsLayout<N, LPB, true, F::R>;
    constexpr int R = F::R, T = F::T;
    constexpr int W = T < 64 ? T : 64;            // lanes of one line within one wave
    constexpr int NW = T / W;                     // waves per line
    __shared__ c32 lds[L::SIZE];
    __shared__ c32 tw[N];
    __shared__ double red[LPB][NW][2];
    stage_twiddles<F>(tw, g.tw[0]);
    const int t = threadIdx.x % T;
    const int l = threadIdx.x / T;
    const int64_t local = (int64_t)blockIdx.x * LPB + l;
    const bool active = local < g.batch;
    const int64_t inst = x.inst_base + (active ? local : 0);
    float2* p = psi + g.offset + (active ? local : 0) * N;

    c32 P[R];
#pragma unroll
    for (int m = 0; m < R; m++) P[m] = active ? p[t + m * T] : make_float2(0.f, 0.f);
    const int64_t line = active ? local : 0;
    double tnow = 0.0;
    double h = active ? x.h[inst] : 1.0;
    int64_t acc = 0, rej = 0;
    bool live = active && tnow < x.t_span && h > 0.0 && isfinite(h);
    __syncthreads();  // twiddles staged
    {
        c32 d[1][R];
#pragma unroll
        for (int m = 0; m < R; m++) d[0][m] = P[m];
        fft_line<F, -1, L, 1>(d, t, l, lds, tw);  // the state in k-space
#pragma unroll
        for (int m = 0; m < R; m++) P[m] = d[0][m];
    }

    // Float copies of the pair's coefficients (the stage weights that vanish are skipped).
    constexpr float b1 = (float)kB5[0], b3 = (float)kB5[2], b4 = (float)kB5[3], b6 = (float)kB5[5];
    constexpr float e1 = (float)(kB5[0] - kB4[0]), e3 = (float)(kB5[2] - kB4[2]), e4 = (float)(kB5[3] - kB4[3]),
                    e5 = (float)(kB5[4] - kB4[4]), e6 = (float)(kB5[5] - kB4[5]);
    while (__syncthreads_or(live ? 1 : 0)) {
        const bool last = tnow + h >= x.t_span;
        const double htry = live ? (last ? x.t_span - tnow : h) : 1e-3;
        const float hf = (float)htry;
        // Stages in order. Only what later stages or the result still need is kept: after
        // the fourth stage the sixth stage's input, the fifth-order sum and the embedded
        // difference are started, and K1..K4 are dropped.
        c32 K1[R], K2[R], K3[R], d[1][R];
#pragma unroll
        for (int m = 0; m < R; m++) d[0][m] = P[m];
        ck_stage<0, CONV, EX, F, L>(d, g, line, t, l, lds, tw, x, htry, hf);
#pragma unroll
        for (int m = 0; m < R; m++) {
            K1[m] = d[0][m];
            d[0][m] = axpy(P[m], kA[1][0], K1[m]);
        }
        ck_stage<1, CONV, EX, F, L>(d, g, line, t, l, lds, tw, x, htry, hf);
#pragma unroll
        for (int m = 0; m < R; m++) {
            K2[m] = d[0][m];
            d[0][m] = axpy(axpy(P[m], kA[2][0], K1[m]), kA[2][1], K2[m]);
        }
        ck_stage<2, CONV, EX, F, L>(d, g, line, t, l, lds, tw, x, htry, hf);
#pragma unroll
        for (int m = 0; m < R; m++) {
            K3[m] = d[0][m];
            d[0][m] = axpy(axpy(axpy(P[m], kA[3][0], K1[m]), kA[3][1], K2[m]), kA[3][2], K3[m]);
        }
        ck_stage<3, CONV, EX, F, L>(d, g, line, t, l, lds, tw, x, htry, hf);
        c32 Y6[R], A[R], D[R];
#pragma unroll
        for (int m = 0; m < R; m++) {
            const c32 k4 = d[0][m];
            d[0][m] = axpy(axpy(axpy(axpy(P[m], kA[4][0], K1[m]), kA[4][1], K2[m]), kA[4][2], K3[m]), kA[4][3], k4);
            Y6[m] = axpy(axpy(axpy(axpy(P[m], kA[5][0], K1[m]), kA[5][1], K2[m]), kA[5][2], K3[m]), kA[5][3], k4);
            A[m] = axpy(axpy(axpy(P[m], b1, K1[m]), b3, K3[m]), b4, k4);
            D[m] = axpy(axpy(make_float2(e1 * K1[m].x, e1 * K1[m].y), e3, K3[m]), e4, k4);
        }
        ck_stage<4, CONV, EX, F, L>(d, g, line, t, l, lds, tw, x, htry, hf);
#pragma unroll
        for (int m = 0; m < R; m++) {
            D[m] = axpy(D[m], e5, d[0][m]);
            d[0][m] = axpy(Y6[m], kA[5][4], d[0][m]);
        }
        ck_stage<5, CONV, EX, F, L>(d, g, line, t, l, lds, tw, x, htry, hf);
        // fifth-order result, embedded difference, and the error estimate: per-thread
        // partials, then a fixed-order sum over the line
        double num = 0.0, den = 0.0;
#pragma unroll
        for (int m = 0; m < R; m++) {
            A[m] = axpy(A[m], b6, d[0][m]);
            D[m] = axpy(D[m], e6, d[0][m]);
            num += (double)fmaf(D[m].x, D[m].x, D[m].y * D[m].y);
            den += (double)fmaf(A[m].x, A[m].x, A[m].y * A[m].y);
        }
#pragma unroll
        for (int o = W / 2; o >= 1; o >>= 1) {
            num += __shfl_xor(num, o, W);
            den += __shfl_xor(den, o, W);
        }
        if (t % W == 0) {
            red[l][t / W][0] = num;
            red[l][t / W][1] = den;
        }
        __syncthreads();
        num = 0.0;
        den = 0.0;
#pragma unroll
        for (int w = 0; w < NW; w++) {
            num += red[l][w][0];
            den += red[l][w][1];
        }
        const double err = sqrt(num / den);
        __syncthreads();  // every line has read its partials before the next step writes them
        if (live) {
            const bool ok = err <= x.tol;
            if (ok) {
                // the fifth-order result moved to t_n + h; the explicit method's result is
                // already there
                if constexpr (!EX) {
                    c32 cs[R];
                    phases<F>(cs, t, x, htry);
                    const float damp = x.gamma != 0.0 ? (float)exp(-x.gamma * htry) : 1.0f;
#pragma unroll
                    for (int m = 0; m < R; m++) A[m] = cmul(A[m], make_float2(damp * cs[m].x, -damp * cs[m].y));
                }
#pragma unroll
                for (int m = 0; m < R; m++) P[m] = A[m];
                if (x.h_log && t == 0 && acc < x.log_cap) x.h_log[inst * x.log_cap + acc] = htry;
                tnow = last ? x.t_span : tnow + htry;
                acc++;
            } else {
                rej++;
            }
            double f;
            if (!isfinite(err)) f = 0.2;
            else if (err == 0.0) f = 5.0;
            else f = fmin(5.0, fmax(0.2, 0.9 * pow(x.tol / err, 0.2)));
            h = htry * f;
            live = tnow < x.t_span && acc + rej < x.max_attempts;
        }
    }
    {
        // back to x-space (every line takes part in the transform's barriers)
        constexpr float inv_n = 1.0f / (float)N;
        c32 d[1][R];
#pragma unroll
        for (int m = 0; m < R; m++) d[0][m] = make_float2(P[m].x * inv_n, P[m].y * inv_n);
        fft_line<F, +1, L, 1>(d, t, l, lds, tw);
#pragma unroll
        for (int m = 0; m < R; m++) P[m] = d[0][m];
    }
    if (!active) return;
    // a line that accepted no step keeps its field as it was, bit for bit
    if (acc > 0) {
#pragma unroll
        for (int m = 0; m < R; m++) p[t + m * T] = P[m];
    }
    if (t == 0) {
        x.h[inst] = h;
        x.stats[3 * inst] = acc;
        x.stats[3 * inst + 1] = rej;
        x.stats[3 * inst + 2] = tnow >= x.t_span ? 1 : 0;
    }
}

template <int N>
static hipError_t go_ark45(const GroupDev& g, float2* psi, const ArkArgs& x, hipStream_t s) {
    constexpr int T = FFTShape<N, 8>::T;
    constexpr int LPB = T >= 64 ? 1 : 64 / T;
    const int64_t blocks = (g.batch + LPB - 1) / LPB;
    const dim3 grid((unsigned)blocks), block(T * LPB);
    if (x.explicit_L) {
        if (g.convK)
            hipLaunchKernelGGL((k_line_ark45<N, LPB, true, true>), grid, block, 0, s, g, psi, x);
        else
            hipLaunchKernelGGL((k_line_ark45<N, LPB, false, true>), grid, block, 0, s, g, psi, x);
    } else {
        if (g.convK)
            hipLaunchKernelGGL((k_line_ark45<N, LPB, true, false>), grid, block, 0, s, g, psi, x);
        else
            hipLaunchKernelGGL((k_line_ark45<N, LPB, false, false>), grid, block, 0, s, g, psi, x);
    }
    return hipGetLastError();
}

hipError_t launch_line_ark45(const GroupDev& g, float2* psi, const ArkArgs& x, hipStream_t s) {
    switch (g.n[0]) {
        case 8: return go_ark45<8>(g, psi, x, s);
        case 16: return go_ark45<16>(g, psi, x, s);
        case 32: return go_ark45<32>(g, psi, x, s);
        case 64: return go_ark45<64>(g, psi, x, s);
        case 128: return go_ark45<128>(g, psi, x, s);
        case 256: return go_ark45<256>(g, psi, x, s);
        case 512: return go_ark45<512>(g, psi, x, s);
        case 1024: return go_ark45<1024>(g, psi, x, s);
        case 2048: return go_ark45<2048>(g, psi, x, s);
        case 4096: return go_ark45<4096>(g, psi, x, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace rk4ip
