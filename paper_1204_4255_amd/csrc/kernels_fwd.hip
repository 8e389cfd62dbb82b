// kernels_fwd.hip -- the 1D whole-line step kernel and the dispatch of the per-axis
// passes (compiled in kernels_pass_*.hip). See pass_common.h for the data flow of a step.
#include "pass_common.h"

namespace rk4ip {

// ---------------------------------------------------------------------------- 1D step

// One workgroup runs LPB whole lines (instances). Every value of the step stays in
// registers; LDS only carries the FFT exchanges. RR values per thread (16 or 8: fewer
// registers and more threads per line). P64: transforms in FP64 (RR = 8), everything
// else as in the complex64 form. SI: the semi-implicit step (one field: a = D psi, the
// midpoint iteration, D(2m - a)) instead of RK4IP.
// EXTRA: the variant with the potential's extra terms (1D groups): the real Wiener
// noise in the potential and the non-local potential. Every G evaluation then needs the
// non-local potential of its whole stage field, so the stages run in phases (one line
// transform pair per G evaluation) instead of point by point.
template <int N, int LPB, bool NOISE, bool P64, int RR, bool SI, bool EXTRA>
__global__ void __launch_bounds__((FFTShape<N, RR>::T * LPB))
    k_line_step(GroupDev g, float2* __restrict__ psi, int nsteps, int64_t step_off,
                const int64_t* __restrict__ step_base) {
    using F = FFTShape<N, RR>;
    using L = LdsLayout<N, LPB, true, F::R>;
    using W = typename std::conditional<P64, c64, c32>::type;  // transform working type
    constexpr int R = F::R, T = F::T;
    __shared__ W lds[2 * L::SIZE];
    __shared__ W tw[N];
    __shared__ W E[N];
    if constexpr (P64)
        stage_tables<F>(tw, E, g.tw64[0], g.E64[0]);
    else
        stage_tables<F>(tw, E, g.tw[0], g.E[0]);
    const int t = threadIdx.x % T;
    const int l = threadIdx.x / T;
    const int64_t inst = (int64_t)blockIdx.x * LPB + l;
    const bool active = inst < g.batch;
    // A cosine or sine group stores the n = N/2 cell centres of a half domain; the line
    // here is its even or odd extension: element e < n is the mirror image of point
    // n - 1 - e (negated for the sine basis), element e >= n is point e - n.
    const int NM = g.basis ? N / 2 : N;
    auto fold = [&](int e, int& j, float& sg) {
        j = e;
        sg = 1.0f;
        if (g.basis) {
            if (e < NM) {
                j = NM - 1 - e;
                if (g.basis == 2) sg = -1.0f;
            } else {
                j = e - NM;
            }
        }
    };
    float2* p = psi + g.offset + inst * NM;

    c32 f[2][R];
    float V[R];
#pragma unroll
    for (int m = 0; m < R; m++) {
        int j;
        float sg;
        fold(t + m * T, j, sg);
        const float2 v0 = active ? p[j] : make_float2(0.f, 0.f);
        f[0][m] = make_float2(sg * v0.x, sg * v0.y);
        float v = trap_V(g, j, 0, 0);
        if (g.Vgrid && active) v += g.Vgrid[inst * NM + j];
        V[m] = v;
    }
    const uint32_t iid = g.id_base + (uint32_t)inst;
    int64_t step = read_step(step_off, step_base);
    __syncthreads();  // tables staged
    for (int s = 0; s < nsteps; s++, step++) {
        if (g.basis && s > 0) {
            // rebuild the mirrored half from the stored half's values, exactly as a reload
            // between launches would: element e < n takes element 2n - 1 - e (the same
            // point), negated for the sine basis (uniform branch)
            c32* xs = reinterpret_cast<c32*>(lds);  // room for LPB lines of N values
            __syncthreads();  // the last step's exchanges are done
#pragma unroll
            for (int m = 0; m < R; m++) {
                const int e = t + m * T;
                if (e >= NM) xs[l * N + e] = f[0][m];
            }
            __syncthreads();
            const float sg = g.basis == 2 ? -1.0f : 1.0f;
#pragma unroll
            for (int m = 0; m < R; m++) {
                const int e = t + m * T;
                if (e < NM) {
                    const c32 v = xs[l * N + (N - 1 - e)];
                    f[0][m] = make_float2(sg * v.x, sg * v.y);
                }
            }
            __syncthreads();  // before this step's transforms reuse the buffer
        }
        c32 nz[R];
#pragma unroll
        for (int m = 0; m < R; m++) {
            if constexpr (NOISE) {
                int j;
                float sg;
                fold(t + m * T, j, sg);
                const float2 z = noise_z(g, j, iid, step);  // odd in the sine basis
                nz[m] = make_float2(sg * (g.noise_c * z.x), sg * (g.noise_c * z.y));
            } else {
                nz[m] = make_float2(0.f, 0.f);
            }
        }
        if constexpr (EXTRA) {
            // potential of this step: V + sigma_V eta, and V_c of each stage field
            float Vs[R], vc[R];
#pragma unroll
            for (int m = 0; m < R; m++) Vs[m] = V[m];
            if constexpr (NOISE) {
                if (g.has_vnoise) {
#pragma unroll
                    for (int m = 0; m < R; m++) {
                        int j;
                        float sg;
                        fold(t + m * T, j, sg);
                        Vs[m] += vnoise(g, j, iid, step);  // a potential: even in both bases
                    }
                }
            }
            const bool conv = g.convK != nullptr;  // uniform
            auto potential = [&](const c32(&x)[R]) {
                if (conv) {
                    conv_V<F, L>(x, vc, t, l, lds, tw, g.convK);
#pragma unroll
                    for (int m = 0; m < R; m++) vc[m] += Vs[m];
                } else {
#pragma unroll
                    for (int m = 0; m < R; m++) vc[m] = Vs[m];
                }
            };
            c32(&f0)[1][R] = *reinterpret_cast<c32(*)[1][R]>(&f[0]);
            if constexpr (SI) {
                propagate<F, L, 1>(f0, t, l, lds, tw, E, false);  // a = D psi
                c32 mid[R];
#pragma unroll
                for (int m = 0; m < R; m++) mid[m] = f[0][m];
                for (int it = 0; it < 3; it++) {
                    potential(mid);
#pragma unroll
                    for (int m = 0; m < R; m++) {
                        const c32 k = hG(g, mid[m], vc[m], nz[m]);
                        mid[m] = make_float2(fmaf(0.5f, k.x, f[0][m].x), fmaf(0.5f, k.y, f[0][m].y));
                    }
                }
#pragma unroll
                for (int m = 0; m < R; m++)
                    f[0][m] = make_float2(fmaf(2.0f, mid[m].x, -f[0][m].x), fmaf(2.0f, mid[m].y, -f[0][m].y));
                propagate<F, L, 1>(f0, t, l, lds, tw, E, false);  // psi' = D(2m - a)
            } else {
                potential(f[0]);
#pragma unroll
                for (int m = 0; m < R; m++) f[1][m] = hG(g, f[0][m], vc[m], nz[m]);
                propagate<F, L, 2>(f, t, l, lds, tw, E, false);  // (a, k1)
                c32 q[R];
#pragma unroll
                for (int m = 0; m < R; m++)
                    q[m] = make_float2(fmaf(0.5f, f[1][m].x, f[0][m].x), fmaf(0.5f, f[1][m].y, f[0][m].y));
                potential(q);
#pragma unroll
                for (int m = 0; m < R; m++) {
                    const c32 k2 = hG(g, q[m], vc[m], nz[m]);
                    // acc so far: a + k1/6 + k2/3 (k1 is not needed after this)
                    f[1][m] = make_float2(f[0][m].x + (f[1][m].x * (1.0f / 6.0f) + k2.x * (1.0f / 3.0f)),
                                          f[0][m].y + (f[1][m].y * (1.0f / 6.0f) + k2.y * (1.0f / 3.0f)));
                    q[m] = make_float2(fmaf(0.5f, k2.x, f[0][m].x), fmaf(0.5f, k2.y, f[0][m].y));
                }
                potential(q);
#pragma unroll
                for (int m = 0; m < R; m++) {
                    const c32 k3 = hG(g, q[m], vc[m], nz[m]);
                    f[0][m] = cadd(f[0][m], k3);  // u = a + k3
                    f[1][m] = make_float2(fmaf(k3.x, 1.0f / 3.0f, f[1][m].x), fmaf(k3.y, 1.0f / 3.0f, f[1][m].y));
                }
                propagate<F, L, 2>(f, t, l, lds, tw, E, false);  // (D u, D acc)
                potential(f[0]);
#pragma unroll
                for (int m = 0; m < R; m++) {
                    const c32 k4 = hG(g, f[0][m], vc[m], nz[m]);
                    f[0][m] = make_float2(fmaf(k4.x, 1.0f / 6.0f, f[1][m].x), fmaf(k4.y, 1.0f / 6.0f, f[1][m].y));
                }
            }
            continue;
        }
        if constexpr (SI) {
            c32(&f0)[1][R] = *reinterpret_cast<c32(*)[1][R]>(&f[0]);
            propagate<F, L, 1>(f0, t, l, lds, tw, E, false);  // a = D psi
#pragma unroll
            for (int m = 0; m < R; m++) {
                const c32 a = f[0][m];
                c32 mid = a;
#pragma unroll
                for (int it = 0; it < 3; it++) {
                    const c32 k = hG(g, mid, V[m], nz[m]);
                    mid = make_float2(fmaf(0.5f, k.x, a.x), fmaf(0.5f, k.y, a.y));
                }
                f[0][m] = make_float2(fmaf(2.0f, mid.x, -a.x), fmaf(2.0f, mid.y, -a.y));
            }
            propagate<F, L, 1>(f0, t, l, lds, tw, E, false);  // psi' = D(2m - a)
            continue;
        }
        // first pair: D psi and D[h G(psi)]
#pragma unroll
        for (int m = 0; m < R; m++) f[1][m] = hG(g, f[0][m], V[m], nz[m]);
        propagate<F, L, 2>(f, t, l, lds, tw, E, false);
        // stages at the midpoint picture
#pragma unroll
        for (int m = 0; m < R; m++) {
            const c32 a = f[0][m], k1 = f[1][m];
            const c32 k2 = hG(g, make_float2(fmaf(0.5f, k1.x, a.x), fmaf(0.5f, k1.y, a.y)), V[m], nz[m]);
            const c32 k3 = hG(g, make_float2(fmaf(0.5f, k2.x, a.x), fmaf(0.5f, k2.y, a.y)), V[m], nz[m]);
            f[0][m] = cadd(a, k3);
            const float sx = k1.x * (1.0f / 6.0f) + (k2.x + k3.x) * (1.0f / 3.0f);
            const float sy = k1.y * (1.0f / 6.0f) + (k2.y + k3.y) * (1.0f / 3.0f);
            f[1][m] = make_float2(a.x + sx, a.y + sy);
        }
        // second pair: D u and D acc
        propagate<F, L, 2>(f, t, l, lds, tw, E, false);
#pragma unroll
        for (int m = 0; m < R; m++) {
            const c32 k4 = hG(g, f[0][m], V[m], nz[m]);
            f[0][m] = make_float2(fmaf(k4.x, 1.0f / 6.0f, f[1][m].x), fmaf(k4.y, 1.0f / 6.0f, f[1][m].y));
        }
    }
    if (active) {
#pragma unroll
        for (int m = 0; m < R; m++) {
            const int e = t + m * T;
            if (g.basis == 0 || e >= NM) p[g.basis ? e - NM : e] = f[0][m];  // the half domain
        }
    }
}

// ---------------------------------------------------------------------------- launchers

int axis_lines(int N, int axis, int n0) { return axis == 0 ? contig_lines(N) : strided_lines(N, n0); }

bool axis_schedule_ok(int N, int mode, int axis, int n0, int lines, int seq, int radix, bool f64, int occ) {
    const bool contig = axis == 0;
    if (!contig && lines > n0) return false;
    switch (N) {
        case 8: return schedule_ok_n<8>(mode, contig, lines, seq, radix, f64, occ);
        case 16: return schedule_ok_n<16>(mode, contig, lines, seq, radix, f64, occ);
        case 32: return schedule_ok_n<32>(mode, contig, lines, seq, radix, f64, occ);
        case 64: return schedule_ok_n<64>(mode, contig, lines, seq, radix, f64, occ);
        case 128: return schedule_ok_n<128>(mode, contig, lines, seq, radix, f64, occ);
        case 256: return schedule_ok_n<256>(mode, contig, lines, seq, radix, f64, occ);
        case 512: return schedule_ok_n<512>(mode, contig, lines, seq, radix, f64, occ);
        case 1024: return schedule_ok_n<1024>(mode, contig, lines, seq, radix, f64, occ);
        default: return false;
    }
}

hipError_t launch_axis(const GroupDev& g, int axis, int mode, const PassArgs& a, hipStream_t s) {
    switch (mode) {
        case PASS_D1:
        case PASS_D2: return launch_axis_d(g, axis, mode, a, s);
        case PASS_FIRST:
        case PASS_LAST2: return launch_axis_first(g, axis, mode, a, s);
        case PASS_LF: return launch_axis_last(g, axis, mode, a, s);
        case PASS_SI: return launch_axis_si(g, axis, a, s);
        case PASS_XF: return launch_axis_xf(g, axis, a, s);
        case PASS_U:
        case PASS_AW:
        case PASS_AS:
        case PASS_AF: return launch_axis_adjoint(g, axis, mode, a, s);
        default: return hipErrorInvalidValue;
    }
}

template <int N, bool P64, int RR, bool SI, bool EXTRA = false>
static hipError_t go_line(const GroupDev& g, float2* psi, int nsteps, int64_t step_off, const int64_t* step_base,
                          hipStream_t s) {
    constexpr int T = FFTShape<N, RR>::T;
    constexpr int LPB = T >= 64 ? 1 : 64 / T;
    const int64_t blocks = (g.batch + LPB - 1) / LPB;
    if (g.has_noise)
        hipLaunchKernelGGL((k_line_step<N, LPB, true, P64, RR, SI, EXTRA>), dim3((unsigned)blocks), dim3(T * LPB), 0, s,
                           g, psi, nsteps, step_off, step_base);
    else
        hipLaunchKernelGGL((k_line_step<N, LPB, false, P64, RR, SI, EXTRA>), dim3((unsigned)blocks), dim3(T * LPB), 0,
                           s, g, psi, nsteps, step_off, step_base);
    return hipGetLastError();
}

template <int N, bool SI>
static hipError_t go_line_p(const GroupDev& g, float2* psi, int nsteps, int64_t step_off, const int64_t* step_base,
                            bool f64, int radix, hipStream_t s) {
    if (g.has_vnoise || g.convK) {
        // the potential's extra terms: 8 values per thread
        if (f64) {
            if constexpr (N <= 2048) return go_line<N, true, 8, SI, true>(g, psi, nsteps, step_off, step_base, s);
            return hipErrorInvalidValue;
        }
        return go_line<N, false, 8, SI, true>(g, psi, nsteps, step_off, step_base, s);
    }
    if (f64) {
        if constexpr (N <= 2048) return go_line<N, true, 8, SI>(g, psi, nsteps, step_off, step_base, s);
        return hipErrorInvalidValue;  // FP64 tables and exchange buffers exceed the LDS
    }
    if (radix == 8) return go_line<N, false, 8, SI>(g, psi, nsteps, step_off, step_base, s);
    if (radix == 0 || radix == 16) return go_line<N, false, 16, SI>(g, psi, nsteps, step_off, step_base, s);
    return hipErrorInvalidValue;
}

template <int N>
static hipError_t go_line_n(const GroupDev& g, float2* psi, int nsteps, int64_t step_off, const int64_t* step_base,
                            bool f64, int radix, bool si, hipStream_t s) {
    if (si) return go_line_p<N, true>(g, psi, nsteps, step_off, step_base, f64, radix, s);
    return go_line_p<N, false>(g, psi, nsteps, step_off, step_base, f64, radix, s);
}

hipError_t launch_line_step(const GroupDev& g, float2* psi, int nsteps, int64_t step_off, const int64_t* step_base,
                            bool f64, int radix, bool semi_implicit, hipStream_t s) {
    switch (g.n[0]) {
        case 8: return go_line_n<8>(g, psi, nsteps, step_off, step_base, f64, radix, semi_implicit, s);
        case 16: return go_line_n<16>(g, psi, nsteps, step_off, step_base, f64, radix, semi_implicit, s);
        case 32: return go_line_n<32>(g, psi, nsteps, step_off, step_base, f64, radix, semi_implicit, s);
        case 64: return go_line_n<64>(g, psi, nsteps, step_off, step_base, f64, radix, semi_implicit, s);
        case 128: return go_line_n<128>(g, psi, nsteps, step_off, step_base, f64, radix, semi_implicit, s);
        case 256: return go_line_n<256>(g, psi, nsteps, step_off, step_base, f64, radix, semi_implicit, s);
        case 512: return go_line_n<512>(g, psi, nsteps, step_off, step_base, f64, radix, semi_implicit, s);
        case 1024: return go_line_n<1024>(g, psi, nsteps, step_off, step_base, f64, radix, semi_implicit, s);
        case 2048: return go_line_n<2048>(g, psi, nsteps, step_off, step_base, f64, radix, semi_implicit, s);
        case 4096: return go_line_n<4096>(g, psi, nsteps, step_off, step_base, f64, radix, semi_implicit, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace rk4ip
