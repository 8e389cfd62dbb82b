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
// One workgroup integrates LPB whole lines, each with its own step: the line, its five
// stored stages and the stage input stay in registers, LDS carries only the FFT
// exchanges and the error-norm partials. e^{L tau} changes with every trial step, so the
// propagator is computed per mode right after the forward transform (phase in FP64,
// reduced to [-pi/2, pi/2] before an FP32 sincos) instead of being read from a table.
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

constexpr double kPiD = 3.14159265358979323846;
constexpr double kInvPiD = 0.31830988618379067154;

}  // namespace

// f <- e^{L tau} f on this thread's R values of its line, in delta form:
// f + F^{-1}[(e^{L tau} - 1)/n F f], with the multiplier of mode m formed from
// theta = alpha k_m^2 tau as (e^{-gamma tau} - 1) - 2 e^{-gamma tau} sin^2(theta/2) and
// -e^{-gamma tau} sin(theta) (no cancellation; theta/2 reduced modulo pi in FP64).
template <class F, class L>
__device__ __forceinline__ void propagate_tau(c32 (&f)[F::R], int t, int l, c32* lds, const c32* tw,
                                              const ArkArgs& x, double tau) {
    constexpr int R = F::R, T = F::T, N = F::NN;
    c32 d[1][R];
#pragma unroll
    for (int m = 0; m < R; m++) d[0][m] = f[m];
    fft_line<F, -1, L, 1>(d, t, l, lds, tw);
    // the damping factor and its distance from 1 (uniform; skipped without damping)
    float damp = 1.0f, em1 = 0.0f;
    if (x.gamma != 0.0) {
        damp = (float)exp(-x.gamma * tau);
        em1 = (float)expm1(-x.gamma * tau);
    }
    constexpr float inv_n = 1.0f / (float)N;  // exact power of two
    const double ph0 = 0.5 * x.alpha * x.kscale * x.kscale * tau;
#pragma unroll
    for (int m = 0; m < R; m++) {
        const int e = t + m * T;
        const double km = (double)(e < N / 2 ? e : e - N);
        const double half = ph0 * km * km;
        const float r = (float)(half - kPiD * rint(half * kInvPiD));
        float s, c;
        sincosf(r, &s, &c);
        const c32 cs = make_float2(fmaf(-2.0f * damp * s, s, em1) * inv_n, -2.0f * damp * s * c * inv_n);
        d[0][m] = cmul(d[0][m], cs);
    }
    fft_line<F, +1, L, 1>(d, t, l, lds, tw);
#pragma unroll
    for (int m = 0; m < R; m++) f[m] = cadd(f[m], d[0][m]);
}

// out = h L v on this thread's R values (the explicit comparison method): transform,
// multiply mode m by h L(k_m) / n = h (-i alpha k_m^2 - gamma) / n, transform back.
template <class F, class L>
__device__ __forceinline__ void apply_hL(const c32 (&v)[F::R], c32 (&out)[F::R], int t, int l, c32* lds,
                                         const c32* tw, const ArkArgs& x, double h) {
    constexpr int R = F::R, T = F::T, N = F::NN;
    c32 d[1][R];
#pragma unroll
    for (int m = 0; m < R; m++) d[0][m] = v[m];
    fft_line<F, -1, L, 1>(d, t, l, lds, tw);
    const double c0 = x.alpha * x.kscale * x.kscale * h / (double)N;
    const float re = (float)(-x.gamma * h / (double)N);
#pragma unroll
    for (int m = 0; m < R; m++) {
        const int e = t + m * T;
        const double km = (double)(e < N / 2 ? e : e - N);
        d[0][m] = cmul(d[0][m], make_float2(re, (float)(-c0 * km * km)));
    }
    fft_line<F, +1, L, 1>(d, t, l, lds, tw);
#pragma unroll
    for (int m = 0; m < R; m++) out[m] = d[0][m];
}

// h G(phi) without noise: -i h (V + g |phi|^2) phi
__device__ __forceinline__ c32 hG_ark(const GroupDev& g, c32 phi, float V, float h) {
    const float m2 = fmaf(phi.x, phi.x, phi.y * phi.y);
    const float w = h * fmaf(g.gnl, m2, V);
    return make_float2(w * phi.y, -w * phi.x);
}

// Stage I (1..5) of a trial step of size h: k_I = e^{-L c_I h} h G(e^{L c_I h} Y_I) with
// Y_I = y + sum_{j<I} a_Ij k_j. A template per stage keeps every index of k a constant,
// so the stages stay in registers.
// EX: the explicit comparison method: the stage input stays in x space and the linear
// part is added to G, k_I = h (L Y_I + G(Y_I)).
template <class F, class L, bool CONV, bool EX>
__device__ __forceinline__ void stage_rhs(c32 (&s)[F::R], const float (&V)[F::R], const GroupDev& g, int t, int l,
                                          c32* lds, const c32* tw, const ArkArgs& x, double h, float hf) {
    c32 lin[F::R];
    if constexpr (EX) apply_hL<F, L>(s, lin, t, l, lds, tw, x, h);
    if constexpr (CONV) {
        // with the non-local potential of the stage field
        float vc[F::R];
        conv_V<F, L>(s, vc, t, l, lds, tw, g.convK);
#pragma unroll
        for (int m = 0; m < F::R; m++) s[m] = hG_ark(g, s[m], V[m] + vc[m], hf);
    } else {
#pragma unroll
        for (int m = 0; m < F::R; m++) s[m] = hG_ark(g, s[m], V[m], hf);
    }
    if constexpr (EX) {
#pragma unroll
        for (int m = 0; m < F::R; m++) s[m] = cadd(s[m], lin[m]);
    }
}

template <int I, bool CONV, bool EX, class F, class L>
__device__ __forceinline__ void ck_stage(c32 (&k)[6][F::R], const c32 (&y)[F::R], const float (&V)[F::R],
                                         const GroupDev& g, int t, int l, c32* lds, const c32* tw,
                                         const ArkArgs& x, double h, float hf) {
#pragma unroll
    for (int m = 0; m < F::R; m++) {
        c32 v = y[m];
#pragma unroll
        for (int j = 0; j < I; j++) v = make_float2(fmaf(kA[I][j], k[j][m].x, v.x), fmaf(kA[I][j], k[j][m].y, v.y));
        k[I][m] = v;
    }
    if constexpr (EX) {
        stage_rhs<F, L, CONV, true>(k[I], V, g, t, l, lds, tw, x, h, hf);
        return;
    }
    propagate_tau<F, L>(k[I], t, l, lds, tw, x, kC[I] * h);  // to the stage time
    stage_rhs<F, L, CONV, false>(k[I], V, g, t, l, lds, tw, x, h, hf);
    propagate_tau<F, L>(k[I], t, l, lds, tw, x, -kC[I] * h);  // back to the picture frame
}

// CONV: G includes the non-local potential (the variant compiled for groups with a kernel).
// EX: the explicit comparison method instead of the interaction picture.
template <int N, int LPB, bool CONV, bool EX>
__global__ void __launch_bounds__((FFTShape<N, 8>::T * LPB))
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

    c32 y[R];
    float V[R];
#pragma unroll
    for (int m = 0; m < R; m++) {
        const int e = t + m * T;
        y[m] = active ? p[e] : make_float2(0.f, 0.f);
        float v = trap_V(g, e, 0, 0);
        if (g.Vgrid && active) v += g.Vgrid[local * N + e];
        V[m] = v;
    }
    double tnow = 0.0;
    double h = active ? x.h[inst] : 1.0;
    int64_t acc = 0, rej = 0;
    bool live = active && tnow < x.t_span && h > 0.0 && isfinite(h);
    __syncthreads();  // twiddles staged

    while (__syncthreads_or(live ? 1 : 0)) {
        const bool last = tnow + h >= x.t_span;
        const double htry = live ? (last ? x.t_span - tnow : h) : 1e-3;
        const float hf = (float)htry;
        c32 k[6][R];
        // stage 1 (c = 0): h G(psi_n)
#pragma unroll
        for (int m = 0; m < R; m++) k[0][m] = y[m];
        stage_rhs<F, L, CONV, EX>(k[0], V, g, t, l, lds, tw, x, htry, hf);
        ck_stage<1, CONV, EX, F, L>(k, y, V, g, t, l, lds, tw, x, htry, hf);
        ck_stage<2, CONV, EX, F, L>(k, y, V, g, t, l, lds, tw, x, htry, hf);
        ck_stage<3, CONV, EX, F, L>(k, y, V, g, t, l, lds, tw, x, htry, hf);
        ck_stage<4, CONV, EX, F, L>(k, y, V, g, t, l, lds, tw, x, htry, hf);
        ck_stage<5, CONV, EX, F, L>(k, y, V, g, t, l, lds, tw, x, htry, hf);
        // fifth-order result and the embedded difference (weights that vanish are skipped)
        c32 y5[R], dl[R];
#pragma unroll
        for (int m = 0; m < R; m++) {
            c32 a = y[m], d = make_float2(0.f, 0.f);
#pragma unroll
            for (int i = 0; i < 6; i++) {
                if (kB5[i] != 0.0) {
                    const float b5 = (float)kB5[i];
                    a = make_float2(fmaf(b5, k[i][m].x, a.x), fmaf(b5, k[i][m].y, a.y));
                }
                if (kB5[i] != kB4[i]) {
                    const float db = (float)(kB5[i] - kB4[i]);
                    d = make_float2(fmaf(db, k[i][m].x, d.x), fmaf(db, k[i][m].y, d.y));
                }
            }
            y5[m] = a;
            dl[m] = d;
        }
        // error estimate: per-thread partials, then a fixed-order sum over the line
        double num = 0.0, den = 0.0;
#pragma unroll
        for (int m = 0; m < R; m++) {
            num += (double)fmaf(dl[m].x, dl[m].x, dl[m].y * dl[m].y);
            den += (double)fmaf(y5[m].x, y5[m].x, y5[m].y * y5[m].y);
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
        // the fifth-order result moved to t_n + h (computed by every line; kept only on
        // acceptance); the explicit method's result is already at t_n + h
        if constexpr (!EX) propagate_tau<F, L>(y5, t, l, lds, tw, x, htry);
        __syncthreads();  // every line has read its partials before the next step writes them
        if (live) {
            const bool ok = err <= x.tol;
            if (ok) {
#pragma unroll
                for (int m = 0; m < R; m++) y[m] = y5[m];
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
    if (!active) return;
#pragma unroll
    for (int m = 0; m < R; m++) p[t + m * T] = y[m];
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
