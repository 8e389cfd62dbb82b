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
    k_line_step(GroupDev g, float2* psi, int nsteps, int64_t step_off,
                const int64_t* __restrict__ step_base, float2* out) {
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
        float2* q = out + g.offset + inst * NM;
#pragma unroll
        for (int m = 0; m < R; m++) {
            const int e = t + m * T;
            if (g.basis == 0 || e >= NM) q[g.basis ? e - NM : e] = f[0][m];  // the half domain
        }
    }
}

// ------------------------------------------------ 1D step, cosine and sine bases

// e^{L h/2} on NF reordered cosine / sine lines in delta form: with V = F v,
// v <- v + F^-1[T1 V + T2 V_rev], V_rev[m] = V[(n - m) mod n], T1 = (A - 1)/n, T2 = B/n (see
// the table builder: A pairs mode m with itself, B with n - m). The pairing is one LDS
// round trip between the transforms; the two products and their sum, which nearly cancel
// on the low modes, are formed in FP64 from FP64 tables and rounded once.
template <class F, class L, int NF>
__device__ __forceinline__ void propagate_pairs(c32 (&f)[NF][F::R], int t, int l, c32* lds, const c32* tw,
                                                const double2* __restrict__ T1, const double2* __restrict__ T2) {
    constexpr int R = F::R, T = F::T, N = F::NN;
    c32 d[NF][R];
#pragma unroll
    for (int q = 0; q < NF; q++)
#pragma unroll
        for (int m = 0; m < R; m++) d[q][m] = f[q][m];
    fft_line<F, -1, L, NF>(d, t, l, lds, tw);
#pragma unroll
    for (int q = 0; q < NF; q++)
#pragma unroll
        for (int m = 0; m < R; m++) lds[q * L::SIZE + L::addr(l, t + m * T)] = d[q][m];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NF; q++)
#pragma unroll
        for (int m = 0; m < R; m++) {
            const int e = t + m * T;
            const c32 rv = lds[q * L::SIZE + L::addr(l, (N - e) & (N - 1))];
            const c64 s = cadd(cmul(widen(d[q][m], c64{}), T1[e]), cmul(widen(rv, c64{}), T2[e]));
            d[q][m] = narrow(s);
        }
    __syncthreads();
    fft_line<F, +1, L, NF>(d, t, l, lds, tw);
#pragma unroll
    for (int q = 0; q < NF; q++)
#pragma unroll
        for (int m = 0; m < R; m++) f[q][m] = cadd(f[q][m], d[q][m]);
}

// The RK4IP (or semi-implicit) step of whole cosine / sine lines of n = N stored points
// through the n-point transform of the reordered line (half the transform length of the
// even / odd extension): element e of a thread's registers is point j(e) = 2e (e < N/2) or
// 2(N - 1 - e) + 1, negated on those odd points in the sine basis. G is pointwise, so the
// stages act on the reordered line as they are; the potential and the noise are those of
// point j(e) (the noise negated with the point in the sine basis). Same data flow as
// k_line_step otherwise, so split runs equal whole runs bitwise.
template <int N, int LPB, bool NOISE, int RR, bool SI>
__global__ void __launch_bounds__((FFTShape<N, RR>::T * LPB))
    k_line_basis(GroupDev g, float2* psi, int nsteps, int64_t step_off,
                 const int64_t* __restrict__ step_base, float2* out) {
    using F = FFTShape<N, RR>;
    using L = LdsLayout<N, LPB, true, F::R>;
    constexpr int R = F::R, T = F::T;
    __shared__ c32 lds[(SI ? 1 : 2) * L::SIZE];
    __shared__ c32 tw[N];
    stage_twiddles<F>(tw, g.tw[0]);
    const double2* __restrict__ T1 = g.pairT1;
    const double2* __restrict__ T2 = g.pairT2;
    const int t = threadIdx.x % T;
    const int l = threadIdx.x / T;
    const int64_t inst = (int64_t)blockIdx.x * LPB + l;
    const bool active = inst < g.batch;
    float2* p = psi + g.offset + inst * N;
    const float odd_sign = g.basis == 2 ? -1.0f : 1.0f;
    auto point = [&](int e) { return e < N / 2 ? 2 * e : 2 * (N - 1 - e) + 1; };
    auto sign = [&](int e) { return e < N / 2 ? 1.0f : odd_sign; };

    c32 f[2][R];
    float V[R];
#pragma unroll
    for (int m = 0; m < R; m++) {
        const int e = t + m * T, j = point(e);
        const float2 v0 = active ? p[j] : make_float2(0.f, 0.f);
        f[0][m] = make_float2(sign(e) * v0.x, sign(e) * v0.y);
        float v = trap_V(g, j, 0, 0);
        if (g.Vgrid && active) v += g.Vgrid[inst * N + j];
        V[m] = v;
    }
    const uint32_t iid = g.id_base + (uint32_t)inst;
    int64_t step = read_step(step_off, step_base);
    __syncthreads();  // twiddles staged
    for (int s = 0; s < nsteps; s++, step++) {
        c32 nz[R];
#pragma unroll
        for (int m = 0; m < R; m++) {
            if constexpr (NOISE) {
                const int e = t + m * T;
                const float2 z = noise_z(g, point(e), iid, step);
                nz[m] = make_float2(sign(e) * (g.noise_c * z.x), sign(e) * (g.noise_c * z.y));
            } else {
                nz[m] = make_float2(0.f, 0.f);
            }
        }
        if constexpr (SI) {
            c32(&f0)[1][R] = *reinterpret_cast<c32(*)[1][R]>(&f[0]);
            propagate_pairs<F, L, 1>(f0, t, l, lds, tw, T1, T2);  // a = D psi
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
            propagate_pairs<F, L, 1>(f0, t, l, lds, tw, T1, T2);  // psi' = D(2m - a)
            continue;
        }
#pragma unroll
        for (int m = 0; m < R; m++) f[1][m] = hG(g, f[0][m], V[m], nz[m]);
        propagate_pairs<F, L, 2>(f, t, l, lds, tw, T1, T2);  // (a, k1)
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
        propagate_pairs<F, L, 2>(f, t, l, lds, tw, T1, T2);  // (D u, D acc)
#pragma unroll
        for (int m = 0; m < R; m++) {
            const c32 k4 = hG(g, f[0][m], V[m], nz[m]);
            f[0][m] = make_float2(fmaf(k4.x, 1.0f / 6.0f, f[1][m].x), fmaf(k4.y, 1.0f / 6.0f, f[1][m].y));
        }
    }
    if (active) {
        float2* q = out + g.offset + inst * N;
#pragma unroll
        for (int m = 0; m < R; m++) {
            const int e = t + m * T;
            q[point(e)] = make_float2(sign(e) * f[0][m].x, sign(e) * f[0][m].y);
        }
    }
}

// ------------------------------------------------------------- 1D step, k-space state

// The same step on a whole 1D Fourier line with its state kept in k-space between the
// steps of a launch: P = F psi (unnormalised). With the picture origin at the midpoint,
// D a = D^2 psi_n, so the RK4 step reads
//     psi_n = F^-1 P / n,  a = F^-1(E P) / n,  k1 = D[h G(psi_n)],
//     k2 = h G(a + k1/2),  k3 = h G(a + k2/2),  k4 = h G(D(a + k3)),
//     P' = E^2 P + E F(k1/6 + k2/3 + k3/3) + F(k4)/6,
// and the semi-implicit step (a = D psi_n, m = a + (h/2) G(m) by three fixed-point
// iterations, psi' = D(2m - a) = D(a + h G(m_2)) with m_2 the second iterate)
//     a = F^-1(E P) / n,  P' = E^2 P + E F(h G(m_2)).
// Both are the steps of the x-space kernel above, regrouped: the field itself is only
// multiplied by E^2 per step and never passes through a transform pair, so the FP32
// rounding of the transforms (their twiddles in particular, whose error is the same every
// step and so adds up linearly) reaches the state only through the stage terms, which
// are of size h G. The transform count is the same (8 per RK4 step, in 6 sequences) or
// halved (2 per semi-implicit step). The state stays in k-space between the launches of
// a run (in the group's buffer g.K: io bit 0 reads it from there, bit 1 leaves it there);
// the first launch of a run transforms psi and the last transforms the state back. The
// rounding of that transform pair is the same every time it is applied (it does not
// shrink with |E - 1| like the propagator's), so it is applied once per run, not per
// launch. Fourier groups without the potential's extra terms, FP32 transforms.
// The two propagator tables are read from global memory where they are used (every
// workgroup reads the same few KB, which stay cached); LDS holds the twiddles and the
// exchange buffers only.
template <int N, int LPB, bool NOISE, int RR, bool SI>
__global__ void __launch_bounds__((FFTShape<N, RR>::T * LPB))
    k_line_kstep(GroupDev g, float2* psi, int nsteps, int64_t step_off,
                 const int64_t* __restrict__ step_base, int io, float2* out) {
    using F = FFTShape<N, RR>;
    using L = LdsLayout<N, LPB, true, F::R>;
    constexpr int R = F::R, T = F::T;
    __shared__ c32 lds[(SI ? 1 : 2) * L::SIZE];
    __shared__ c32 tw[N];
    stage_twiddles<F>(tw, g.tw[0]);
    const float2* __restrict__ E1 = g.E[0];  // (E - 1)/n
    const float2* __restrict__ E2 = g.E2;    // (E^2 - 1)/n
    const int t = threadIdx.x % T;
    const int l = threadIdx.x / T;
    const int64_t inst = (int64_t)blockIdx.x * LPB + l;
    const bool active = inst < g.batch;
    float2* p = psi + g.offset + inst * N;
    float2* kp = g.K + inst * N;
    const float fn = (float)N, inv_n = g.inv_n[0];  // exact powers of two
    const c32 zero = make_float2(0.f, 0.f);

    c32 P[1][R];
    float V[R];
#pragma unroll
    for (int m = 0; m < R; m++) {
        const int j = t + m * T;
        P[0][m] = active ? ((io & 1) ? kp[j] : p[j]) : zero;
        float v = trap_V(g, j, 0, 0);
        if (g.Vgrid && active) v += g.Vgrid[inst * N + j];
        V[m] = v;
    }
    const uint32_t iid = g.id_base + (uint32_t)inst;
    int64_t step = read_step(step_off, step_base);
    __syncthreads();  // tables staged
    if (!(io & 1)) fft_line<F, -1, L, 1>(P, t, l, lds, tw);  // P = F psi (uniform branch)
    // E^q z = z + n ((E^q - 1)/n) z for a k-space value z at element j
    auto mulE = [&](c32 z, int j) { return cadd(z, cmul(z, cscale(E1[j], fn))); };
    for (int s = 0; s < nsteps; s++, step++) {
        c32 nz[R];
        if constexpr (NOISE) {
            if (T >= 2 && g.noise_sub == 1) {
                // lanes t and t ^ 1 hold the pairs of points one Philox block feeds (uniform)
                noise_z_pairs<R>(g, t, T, iid, step, nz);
            } else {
#pragma unroll
                for (int m = 0; m < R; m++) nz[m] = noise_z(g, t + m * T, iid, step);
            }
#pragma unroll
            for (int m = 0; m < R; m++) nz[m] = make_float2(g.noise_c * nz[m].x, g.noise_c * nz[m].y);
        } else {
#pragma unroll
            for (int m = 0; m < R; m++) nz[m] = zero;
        }
        c32 inc[1][R];  // F of the step's increment, without E^2 P
        if constexpr (SI) {
            c32 x[1][R];
#pragma unroll
            for (int m = 0; m < R; m++) x[0][m] = mulE(P[0][m], t + m * T);
            fft_line<F, +1, L, 1>(x, t, l, lds, tw);
#pragma unroll
            for (int m = 0; m < R; m++) {
                const c32 a = cscale(x[0][m], inv_n);
                c32 mid = a;
#pragma unroll
                for (int it = 0; it < 2; it++) {
                    const c32 k = hG(g, mid, V[m], nz[m]);
                    mid = make_float2(fmaf(0.5f, k.x, a.x), fmaf(0.5f, k.y, a.y));
                }
                inc[0][m] = hG(g, mid, V[m], nz[m]);  // 2 (m_3 - a)
            }
            fft_line<F, -1, L, 1>(inc, t, l, lds, tw);
#pragma unroll
            for (int m = 0; m < R; m++) inc[0][m] = mulE(inc[0][m], t + m * T);
        } else {
            // psi_n and a = D psi_n from the state
            c32 x[2][R];
#pragma unroll
            for (int m = 0; m < R; m++) {
                x[0][m] = P[0][m];
                x[1][m] = mulE(P[0][m], t + m * T);
            }
            fft_line<F, +1, L, 2>(x, t, l, lds, tw);
            // k1 = D[h G(psi_n)] (delta form)
            c32 k1[1][R];
#pragma unroll
            for (int m = 0; m < R; m++) {
                x[0][m] = cscale(x[0][m], inv_n);  // psi_n
                x[1][m] = cscale(x[1][m], inv_n);  // a
                k1[0][m] = hG(g, x[0][m], V[m], nz[m]);
            }
            propagate<F, L, 1>(k1, t, l, lds, tw, E1, false);
            // stages: u = a + k3 in x[0], c = k1/6 + k2/3 + k3/3 in x[1]
#pragma unroll
            for (int m = 0; m < R; m++) {
                const c32 a = x[1][m], q1 = k1[0][m];
                const c32 k2 = hG(g, make_float2(fmaf(0.5f, q1.x, a.x), fmaf(0.5f, q1.y, a.y)), V[m], nz[m]);
                const c32 k3 = hG(g, make_float2(fmaf(0.5f, k2.x, a.x), fmaf(0.5f, k2.y, a.y)), V[m], nz[m]);
                x[0][m] = cadd(a, k3);
                x[1][m] = make_float2(q1.x * (1.0f / 6.0f) + (k2.x + k3.x) * (1.0f / 3.0f),
                                      q1.y * (1.0f / 6.0f) + (k2.y + k3.y) * (1.0f / 3.0f));
            }
            fft_line<F, -1, L, 2>(x, t, l, lds, tw);  // (F u, F c)
            // w = D u = F^-1(E F u)/n, k4 = h G(w)
            c32 w[1][R];
#pragma unroll
            for (int m = 0; m < R; m++) w[0][m] = mulE(x[0][m], t + m * T);
            fft_line<F, +1, L, 1>(w, t, l, lds, tw);
#pragma unroll
            for (int m = 0; m < R; m++) inc[0][m] = hG(g, cscale(w[0][m], inv_n), V[m], nz[m]);
            fft_line<F, -1, L, 1>(inc, t, l, lds, tw);  // F k4
#pragma unroll
            for (int m = 0; m < R; m++) {
                const c32 Ec = mulE(x[1][m], t + m * T);
                inc[0][m] = make_float2(fmaf(inc[0][m].x, 1.0f / 6.0f, Ec.x), fmaf(inc[0][m].y, 1.0f / 6.0f, Ec.y));
            }
        }
        // P' = E^2 P + increment = P + (n (E^2 - 1)/n P + increment)
#pragma unroll
        for (int m = 0; m < R; m++) {
            const c32 d = cmul(P[0][m], cscale(E2[t + m * T], fn));
            P[0][m] = cadd(P[0][m], cadd(d, inc[0][m]));
        }
    }
    if (io & 2) {
        if (active) {
#pragma unroll
            for (int m = 0; m < R; m++) kp[t + m * T] = P[0][m];
        }
        return;
    }
    fft_line<F, +1, L, 1>(P, t, l, lds, tw);  // back to x-space
    if (active) {
        float2* q = out + g.offset + inst * N;
#pragma unroll
        for (int m = 0; m < R; m++) q[t + m * T] = cscale(P[0][m], inv_n);
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
        case PASS_AS:
        case PASS_AF:
        case PASS_D2U:
        case PASS_XAW: return launch_axis_adjoint(g, axis, mode, a, s);
        default: return hipErrorInvalidValue;
    }
}

template <int N, bool P64, int RR, bool SI, bool EXTRA = false>
static hipError_t go_line(const GroupDev& g, float2* psi, int nsteps, int64_t step_off, const int64_t* step_base,
                          float2* out, hipStream_t s) {
    constexpr int T = FFTShape<N, RR>::T;
    constexpr int LPB = T >= 64 ? 1 : 64 / T;
    const int64_t blocks = (g.batch + LPB - 1) / LPB;
    if (g.has_noise)
        hipLaunchKernelGGL((k_line_step<N, LPB, true, P64, RR, SI, EXTRA>), dim3((unsigned)blocks), dim3(T * LPB), 0, s,
                           g, psi, nsteps, step_off, step_base, out);
    else
        hipLaunchKernelGGL((k_line_step<N, LPB, false, P64, RR, SI, EXTRA>), dim3((unsigned)blocks), dim3(T * LPB), 0,
                           s, g, psi, nsteps, step_off, step_base, out);
    return hipGetLastError();
}

template <int N, int RR, bool SI>
static hipError_t go_kline(const GroupDev& g, float2* psi, int nsteps, int64_t step_off, const int64_t* step_base,
                           int io, float2* out, hipStream_t s) {
    constexpr int T = FFTShape<N, RR>::T;
    constexpr int LPB = T >= 64 ? 1 : 64 / T;
    const int64_t blocks = (g.batch + LPB - 1) / LPB;
    if (g.has_noise)
        hipLaunchKernelGGL((k_line_kstep<N, LPB, true, RR, SI>), dim3((unsigned)blocks), dim3(T * LPB), 0, s, g, psi,
                           nsteps, step_off, step_base, io, out);
    else
        hipLaunchKernelGGL((k_line_kstep<N, LPB, false, RR, SI>), dim3((unsigned)blocks), dim3(T * LPB), 0, s, g, psi,
                           nsteps, step_off, step_base, io, out);
    return hipGetLastError();
}

template <int N, int RR, bool SI>
static hipError_t go_basis(const GroupDev& g, float2* psi, int nsteps, int64_t step_off, const int64_t* step_base,
                           float2* out, hipStream_t s) {
    constexpr int T = FFTShape<N, RR>::T;
    constexpr int LPB = T >= 64 ? 1 : 64 / T;
    const int64_t blocks = (g.batch + LPB - 1) / LPB;
    if (g.has_noise)
        hipLaunchKernelGGL((k_line_basis<N, LPB, true, RR, SI>), dim3((unsigned)blocks), dim3(T * LPB), 0, s, g, psi,
                           nsteps, step_off, step_base, out);
    else
        hipLaunchKernelGGL((k_line_basis<N, LPB, false, RR, SI>), dim3((unsigned)blocks), dim3(T * LPB), 0, s, g, psi,
                           nsteps, step_off, step_base, out);
    return hipGetLastError();
}

template <int N, bool SI>
static hipError_t go_line_p(const GroupDev& g, float2* psi, int nsteps, int64_t step_off, const int64_t* step_base,
                            bool f64, int radix, int io, float2* out, hipStream_t s) {
    if (g.basis && g.pairT1) {
        // a cosine / sine line through its reordered n-point transform
        if (f64 || g.has_vnoise || io) return hipErrorInvalidValue;
        if (radix == 8) return go_basis<N, 8, SI>(g, psi, nsteps, step_off, step_base, out, s);
        if (radix == 0 || radix == 16) return go_basis<N, 16, SI>(g, psi, nsteps, step_off, step_base, out, s);
        return hipErrorInvalidValue;
    }
    if (g.K) {
        // Fourier lines with a k-space state buffer: the step with the state in k-space
        if (f64 || g.basis || g.has_vnoise || g.convK || !g.E2) return hipErrorInvalidValue;
        if (radix == 8) return go_kline<N, 8, SI>(g, psi, nsteps, step_off, step_base, io, out, s);
        if (radix == 0 || radix == 16) return go_kline<N, 16, SI>(g, psi, nsteps, step_off, step_base, io, out, s);
        return hipErrorInvalidValue;
    }
    if (io) return hipErrorInvalidValue;  // no k-space state to read or keep
    if (g.has_vnoise || g.convK) {
        // the potential's extra terms: 8 values per thread
        if (f64) {
            if constexpr (N <= 2048) return go_line<N, true, 8, SI, true>(g, psi, nsteps, step_off, step_base, out, s);
            return hipErrorInvalidValue;
        }
        return go_line<N, false, 8, SI, true>(g, psi, nsteps, step_off, step_base, out, s);
    }
    if (f64) {
        if constexpr (N <= 2048) return go_line<N, true, 8, SI>(g, psi, nsteps, step_off, step_base, out, s);
        return hipErrorInvalidValue;  // FP64 tables and exchange buffers exceed the LDS
    }
    if (radix == 8) return go_line<N, false, 8, SI>(g, psi, nsteps, step_off, step_base, out, s);
    if (radix == 0 || radix == 16) return go_line<N, false, 16, SI>(g, psi, nsteps, step_off, step_base, out, s);
    return hipErrorInvalidValue;
}

template <int N>
static hipError_t go_line_n(const GroupDev& g, float2* psi, int nsteps, int64_t step_off, const int64_t* step_base,
                            bool f64, int radix, bool si, int io, float2* out, hipStream_t s) {
    if (si) return go_line_p<N, true>(g, psi, nsteps, step_off, step_base, f64, radix, io, out, s);
    return go_line_p<N, false>(g, psi, nsteps, step_off, step_base, f64, radix, io, out, s);
}

hipError_t launch_line_step(const GroupDev& g, float2* psi, int nsteps, int64_t step_off, const int64_t* step_base,
                            bool f64, int radix, bool semi_implicit, hipStream_t s, int io, float2* out) {
    if (!out) out = psi;
    if (out != psi && (io & 2)) return hipErrorInvalidValue;  // the state stays in K
    switch (g.n[0]) {
        case 8: return go_line_n<8>(g, psi, nsteps, step_off, step_base, f64, radix, semi_implicit, io, out, s);
        case 16: return go_line_n<16>(g, psi, nsteps, step_off, step_base, f64, radix, semi_implicit, io, out, s);
        case 32: return go_line_n<32>(g, psi, nsteps, step_off, step_base, f64, radix, semi_implicit, io, out, s);
        case 64: return go_line_n<64>(g, psi, nsteps, step_off, step_base, f64, radix, semi_implicit, io, out, s);
        case 128: return go_line_n<128>(g, psi, nsteps, step_off, step_base, f64, radix, semi_implicit, io, out, s);
        case 256: return go_line_n<256>(g, psi, nsteps, step_off, step_base, f64, radix, semi_implicit, io, out, s);
        case 512: return go_line_n<512>(g, psi, nsteps, step_off, step_base, f64, radix, semi_implicit, io, out, s);
        case 1024: return go_line_n<1024>(g, psi, nsteps, step_off, step_base, f64, radix, semi_implicit, io, out, s);
        case 2048: return go_line_n<2048>(g, psi, nsteps, step_off, step_base, f64, radix, semi_implicit, io, out, s);
        case 4096: return go_line_n<4096>(g, psi, nsteps, step_off, step_base, f64, radix, semi_implicit, io, out, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace rk4ip
