// kernels_adj.hip -- adjoint-step kernels (not in the paper): the per-axis passes D2U,
// XAW, AS, AF and the 1D whole-line adjoint step.
#include "pass_common.h"

namespace rk4ip {

// ---------------------------------------------------------------------------- 1D adjoint step

// Adjoint of one step of LPB whole lines: forward stages recomputed from psi_n in
// registers, then the two transposed D-pairs; lam (in/out) is the adjoint state and vbar
// accumulates the potential gradient.
template <int N, int LPB>
__global__ void __launch_bounds__(FFTShape<N>::T* LPB)
    k_line_adjoint(GroupDev g, const float2* __restrict__ psi_n, float2* __restrict__ lam, double* __restrict__ vbar,
                   int64_t step_off, const int64_t* __restrict__ step_base) {
    const int64_t step = read_step(step_off, step_base);
    using F = FFTShape<N>;
    using L = LdsLayout<N, LPB, true, F::R>;
    constexpr int R = F::R, T = F::T;
    __shared__ c32 lds[2 * L::SIZE];
    __shared__ c32 tw[N];
    __shared__ float2 E[N];
    stage_tables<F>(tw, E, g.tw[0], g.E[0]);
    const int t = threadIdx.x % T;
    const int l = threadIdx.x / T;
    const int64_t inst = (int64_t)blockIdx.x * LPB + l;
    const bool active = inst < g.batch;
    const int64_t base = g.offset + (active ? inst : 0) * N;
    const uint32_t iid = g.id_base + (uint32_t)inst;
    const c32 zero = make_float2(0.f, 0.f);
    auto V_at = [&](int m) {
        float v = trap_V(g, t + m * T, 0, 0);
        if (g.Vgrid && active) v += g.Vgrid[inst * N + t + m * T];
        return v;
    };
    auto nz_at = [&](int m) {
        if (!g.has_noise) return zero;
        const float2 z = noise_z(g, t + m * T, iid, step);
        return make_float2(g.noise_c * z.x, g.noise_c * z.y);
    };
    __syncthreads();  // tables staged
    // forward: (a, k1) = D (psi, hG(psi))
    c32 f[2][R];
#pragma unroll
    for (int m = 0; m < R; m++) {
        f[0][m] = active ? psi_n[base + t + m * T] : zero;
        f[1][m] = hG(g, f[0][m], V_at(m), nz_at(m));
    }
    propagate<F, L, 2>(f, t, l, lds, tw, E, false);
    // w = D(a + k3): keep (a, k1) in f, the transform of u in w[0]
    c32 w[1][R];
#pragma unroll
    for (int m = 0; m < R; m++) {
        const c32 a = f[0][m], k1 = f[1][m];
        const float V = V_at(m);
        const c32 nz = nz_at(m);
        const c32 k2 = hG(g, make_float2(fmaf(0.5f, k1.x, a.x), fmaf(0.5f, k1.y, a.y)), V, nz);
        const c32 k3 = hG(g, make_float2(fmaf(0.5f, k2.x, a.x), fmaf(0.5f, k2.y, a.y)), V, nz);
        w[0][m] = cadd(a, k3);
    }
    propagate<F, L, 1>(w, t, l, lds, tw, E, false);
    // adjoint: (lam, wbar) -> D^T -> (accbar, ubar)
    c32 b[2][R];
    float vacc[R];
#pragma unroll
    for (int m = 0; m < R; m++) {
        const c32 lm = active ? lam[base + t + m * T] : zero;
        const c32 k4b = cscale(lm, 1.0f / 6.0f);
        b[0][m] = lm;
        b[1][m] = hJT(g, w[0][m], V_at(m), k4b);
        vacc[m] = hImconj(g, k4b, w[0][m]);
    }
    propagate<F, L, 2>(b, t, l, lds, tw, E, true);
#pragma unroll
    for (int m = 0; m < R; m++) {
        const float V = V_at(m);
        const c32 nz = nz_at(m);
        const c32 a = f[0][m], k1 = f[1][m];
        const c32 p2 = make_float2(fmaf(0.5f, k1.x, a.x), fmaf(0.5f, k1.y, a.y));
        const c32 k2 = hG(g, p2, V, nz);
        const c32 p3 = make_float2(fmaf(0.5f, k2.x, a.x), fmaf(0.5f, k2.y, a.y));
        const c32 accb = b[0][m], ub = b[1][m];
        const c32 k3b = make_float2(fmaf(accb.x, 1.0f / 3.0f, ub.x), fmaf(accb.y, 1.0f / 3.0f, ub.y));
        const c32 p3b = hJT(g, p3, V, k3b);
        const c32 k2b = make_float2(fmaf(accb.x, 1.0f / 3.0f, 0.5f * p3b.x), fmaf(accb.y, 1.0f / 3.0f, 0.5f * p3b.y));
        const c32 p2b = hJT(g, p2, V, k2b);
        const c32 k1b = make_float2(fmaf(accb.x, 1.0f / 6.0f, 0.5f * p2b.x), fmaf(accb.y, 1.0f / 6.0f, 0.5f * p2b.y));
        vacc[m] += hImconj(g, k3b, p3) + hImconj(g, k2b, p2);
        b[0][m] = make_float2(accb.x + ub.x + p3b.x + p2b.x, accb.y + ub.y + p3b.y + p2b.y);
        b[1][m] = k1b;
    }
    propagate<F, L, 2>(b, t, l, lds, tw, E, true);
    if (!active) return;
#pragma unroll
    for (int m = 0; m < R; m++) {
        const c32 pn = psi_n[base + t + m * T];
        const c32 r = hJT(g, pn, V_at(m), b[1][m]);
        vacc[m] += hImconj(g, b[1][m], pn);
        lam[base + t + m * T] = cadd(b[0][m], r);
        if (vbar) vbar[base + t + m * T] += (double)vacc[m];
    }
}

__global__ void k_vbar_to_float(const double* __restrict__ v, float* __restrict__ out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)v[i];
}

// ---------------------------------------------------------------------------- launchers

hipError_t launch_axis_adjoint(const GroupDev& g, int axis, int mode, const PassArgs& a, hipStream_t s) {
    switch (mode) {
        case PASS_AS: return go_axis_mode<PASS_AS>(g, axis, a, s);
        case PASS_AF: return go_axis_mode<PASS_AF>(g, axis, a, s);
        case PASS_D2U: return go_axis_mode<PASS_D2U>(g, axis, a, s);
        case PASS_XAW: return go_axis_mode<PASS_XAW>(g, axis, a, s);
        default: return hipErrorInvalidValue;
    }
}

template <int N>
static hipError_t go_line_adj(const GroupDev& g, const float2* psi_n, float2* lam, double* vbar, int64_t step,
                              const int64_t* step_base, hipStream_t s) {
    constexpr int T = FFTShape<N>::T;
    constexpr int LPB = T >= 64 ? 1 : 64 / T;
    const int64_t blocks = (g.batch + LPB - 1) / LPB;
    hipLaunchKernelGGL((k_line_adjoint<N, LPB>), dim3((unsigned)blocks), dim3(T * LPB), 0, s, g, psi_n, lam, vbar,
                       step, step_base);
    return hipGetLastError();
}

hipError_t launch_line_adjoint(const GroupDev& g, const float2* psi_n, float2* lam, double* vbar, int64_t step,
                               const int64_t* step_base, hipStream_t s) {
    switch (g.n[0]) {
        case 8: return go_line_adj<8>(g, psi_n, lam, vbar, step, step_base, s);
        case 16: return go_line_adj<16>(g, psi_n, lam, vbar, step, step_base, s);
        case 32: return go_line_adj<32>(g, psi_n, lam, vbar, step, step_base, s);
        case 64: return go_line_adj<64>(g, psi_n, lam, vbar, step, step_base, s);
        case 128: return go_line_adj<128>(g, psi_n, lam, vbar, step, step_base, s);
        case 256: return go_line_adj<256>(g, psi_n, lam, vbar, step, step_base, s);
        case 512: return go_line_adj<512>(g, psi_n, lam, vbar, step, step_base, s);
        case 1024: return go_line_adj<1024>(g, psi_n, lam, vbar, step, step_base, s);
        case 2048: return go_line_adj<2048>(g, psi_n, lam, vbar, step, step_base, s);
        case 4096: return go_line_adj<4096>(g, psi_n, lam, vbar, step, step_base, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_vbar_to_float(const double* vbar, float* out, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_vbar_to_float, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, vbar, out, n);
    return hipGetLastError();
}

}  // namespace rk4ip
