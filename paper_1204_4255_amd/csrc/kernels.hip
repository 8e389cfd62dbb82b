// kernels.hip -- gfx950 kernels of the RK4IP step and their launchers.
//
// The step (Dennis, Hope & Johnsson, arXiv:1204.4255: classic RK4, Sec. 3.5, in the
// interaction picture of Sec. 3.6 with the picture origin at the step midpoint) is
//   a  = D psi,   k1 = D[h G(psi)],   k2 = h G(a + k1/2),   k3 = h G(a + k2/2),
//   k4 = h G(D(a + k3)),   psi' = D(a + k1/6 + k2/3 + k3/3) + k4/6,
// with D = e^{L h/2} applied per lattice axis (Sec. 3.2 factorisation): FFT along the
// axis, multiply by e^{L_a h/2}, inverse FFT. The four D applications come in two pairs
// of two fields, so on a 2D/3D lattice a step is two sweeps over the axes, each pass
// reading and writing two complex64 fields once:
//   FIRST (axis 0):   psi            -> (psi, hG(psi)) -> D_0 -> (A, B)
//   D2    (middle):   (A, B)         -> D_a            -> (A, B)
//   LAST1 (last axis):(A, B)         -> D_a -> a, k1; k2, k3; u = a + k3,
//                                        acc = a + k1/6 + k2/3 + k3/3 -> (A, B) = (u, acc)
//   D2    (axis 0, middle axes)
//   LAST2 (last axis):(A, B)         -> D_a -> psi' = D acc + hG(D u)/6 -> psi
// A 1D line fits one workgroup, so the whole step (eight transforms) runs in registers
// and LDS with one read and one write of psi (k_line_step), optionally for several
// steps per launch.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"
#include "launch.h"

namespace rk4ip {

// ---------------------------------------------------------------------------- helpers

__device__ __forceinline__ int64_t read_step(int64_t step_off, const int64_t* step_base) {
    return step_off + (step_base ? *step_base : 0);
}

// D_a on NF lines held in registers, in delta form: f <- f + F^{-1}[(E_a - 1)/n F f]
// (adj: the transpose, with the conjugate multiplier). All threads of the block call it.
template <int N, class L, int NF>
__device__ __forceinline__ void propagate(c32 (&f)[NF][FFTShape<N>::R], int t, int l, c32* lds,
                                          const c32* __restrict__ tw, const float2* __restrict__ E, bool adj) {
    using F = FFTShape<N>;
    c32 o[NF][F::R];
#pragma unroll
    for (int q = 0; q < NF; q++)
#pragma unroll
        for (int m = 0; m < F::R; m++) o[q][m] = f[q][m];
    fft_line<N, -1, L, NF>(f, t, l, lds, tw);
#pragma unroll
    for (int m = 0; m < F::R; m++) {
        float2 cs = E[t + m * F::T];
        if (adj) cs.y = -cs.y;
#pragma unroll
        for (int q = 0; q < NF; q++) f[q][m] = cmul(f[q][m], cs);
    }
    fft_line<N, +1, L, NF>(f, t, l, lds, tw);
#pragma unroll
    for (int q = 0; q < NF; q++)
#pragma unroll
        for (int m = 0; m < F::R; m++) f[q][m] = cadd(f[q][m], o[q][m]);
}

__global__ void k_counter(int64_t* c, int64_t v, int add) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *c = add ? *c + v : v;
}

// ---------------------------------------------------------------------------- debug

__global__ void k_philox(uint32_t k0, uint32_t k1, const uint4* __restrict__ ctr, int64_t n, uint4* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint4 c = ctr[i];
    U4 u = {c.x, c.y, c.z, c.w};
    const U4 r = philox4x32_10(u, k0, k1);
    out[i] = make_uint4(r.x, r.y, r.z, r.w);
}

__global__ void k_noise(GroupDev g, int64_t step, float2* __restrict__ xi) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.batch * g.M) return;
    const int64_t b = i / g.M;
    const int64_t j = i - b * g.M;
    const float2 z = noise_z(g, j, g.id_base + (uint32_t)b, step);
    xi[i] = make_float2(g.xi_scale * z.x, g.xi_scale * z.y);
}

template <int N, int LINES>
__global__ void __launch_bounds__(FFTShape<N>::T* LINES)
    k_fft_lines(const float2* __restrict__ in, float2* __restrict__ out, int64_t nlines, int sign,
                const float2* __restrict__ tw) {
    using F = FFTShape<N>;
    using L = LdsLayout<N, LINES, true>;
    __shared__ c32 lds[L::SIZE];
    const int t = threadIdx.x % F::T;
    const int l = threadIdx.x / F::T;
    const int64_t line = (int64_t)blockIdx.x * LINES + l;
    const bool active = line < nlines;
    c32 v[1][F::R];
#pragma unroll
    for (int m = 0; m < F::R; m++) v[0][m] = active ? in[line * N + t + m * F::T] : make_float2(0.f, 0.f);
    if (sign < 0)
        fft_line<N, -1, L, 1>(v, t, l, lds, tw);
    else
        fft_line<N, +1, L, 1>(v, t, l, lds, tw);
    if (active) {
#pragma unroll
        for (int m = 0; m < F::R; m++) out[line * N + t + m * F::T] = v[0][m];
    }
}

// ---------------------------------------------------------------------------- 1D step

// One workgroup runs LPB whole lines (instances). Every value of the step stays in
// registers; LDS only carries the FFT exchanges.
template <int N, int LPB>
__global__ void __launch_bounds__(FFTShape<N>::T* LPB)
    k_line_step(GroupDev g, float2* __restrict__ psi, int nsteps, int64_t step_off,
                const int64_t* __restrict__ step_base) {
    using F = FFTShape<N>;
    using L = LdsLayout<N, LPB, true>;
    constexpr int R = F::R, T = F::T;
    __shared__ c32 lds[2 * L::SIZE];
    const int t = threadIdx.x % T;
    const int l = threadIdx.x / T;
    const int64_t inst = (int64_t)blockIdx.x * LPB + l;
    const bool active = inst < g.batch;
    float2* p = psi + g.offset + inst * N;
    const float2* __restrict__ E = g.E[0];
    const float2* __restrict__ tw = g.tw[0];

    c32 f[2][R];
    float V[R];
#pragma unroll
    for (int m = 0; m < R; m++) {
        const int e = t + m * T;
        f[0][m] = active ? p[e] : make_float2(0.f, 0.f);
        float v = trap_V(g, e, 0, 0);
        if (g.Vgrid && active) v += g.Vgrid[inst * N + e];
        V[m] = v;
    }
    const uint32_t iid = g.id_base + (uint32_t)inst;
    int64_t step = read_step(step_off, step_base);
    for (int s = 0; s < nsteps; s++, step++) {
        c32 nz[R];
#pragma unroll
        for (int m = 0; m < R; m++) {
            if (g.has_noise) {
                const float2 z = noise_z(g, t + m * T, iid, step);
                nz[m] = make_float2(g.noise_c * z.x, g.noise_c * z.y);
            } else {
                nz[m] = make_float2(0.f, 0.f);
            }
        }
        // first pair: D psi and D[h G(psi)]
#pragma unroll
        for (int m = 0; m < R; m++) f[1][m] = hG(g, f[0][m], V[m], nz[m]);
        propagate<N, L, 2>(f, t, l, lds, tw, E, false);
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
        propagate<N, L, 2>(f, t, l, lds, tw, E, false);
#pragma unroll
        for (int m = 0; m < R; m++) {
            const c32 k4 = hG(g, f[0][m], V[m], nz[m]);
            f[0][m] = make_float2(fmaf(k4.x, 1.0f / 6.0f, f[1][m].x), fmaf(k4.y, 1.0f / 6.0f, f[1][m].y));
        }
    }
    if (active) {
#pragma unroll
        for (int m = 0; m < R; m++) p[t + m * T] = f[0][m];
    }
}

// ---------------------------------------------------------------------------- axis passes

// Which lines a workgroup owns and where element e of its line l lives.
// CONTIG: LINES consecutive lines along axis 0 (threads of a line are adjacent lanes).
// strided: LINES adjacent x columns of one (instance, outer index) along axis 1 or 2
// (adjacent lanes hold adjacent columns, so each row segment is one coalesced access).
// Addresses are a workgroup-uniform 64-bit tile base plus 32-bit per-thread offsets,
// shared by every field the pass touches.
template <int N, bool CONTIG, int LINES>
struct Tile {
    int64_t base;      // uniform: group-relative point index of the tile origin
    uint32_t off0;     // this thread's element 0 relative to base
    uint32_t dstep;    // offset between element t + m T and t + (m+1) T
    int64_t inst;      // instance of this thread's line
    int64_t jbase;     // in-instance index of this thread's element 0 (noise counter, Vgrid)
    uint32_t jstride;  // in-instance index step per element along the axis
    bool active;

    __device__ __forceinline__ Tile(const GroupDev& g, int axis, int l, int t) {
        constexpr int T = FFTShape<N>::T;
        if constexpr (CONTIG) {
            const int64_t lines_per_inst = g.M >> g.log2n[0];
            const int64_t nlines = g.batch * lines_per_inst;
            const int64_t line = (int64_t)blockIdx.x * LINES + l;
            active = line < nlines;
            const int64_t ln = active ? line : 0;
            base = (int64_t)blockIdx.x * LINES * N;
            off0 = (uint32_t)(l * N + t);
            dstep = T;
            inst = ln / lines_per_inst;
            jbase = (ln - inst * lines_per_inst) * N + t;
            jstride = 1;
        } else {
            const int xt_count = g.n[0] / LINES;
            const int outer_n = (axis == 1) ? g.n[2] : g.n[1];
            int64_t bid = blockIdx.x;
            const int xt = (int)(bid % xt_count);
            bid /= xt_count;
            const int outer = (int)(bid % outer_n);
            inst = bid / outer_n;
            active = true;
            const uint32_t stride = (axis == 1) ? (uint32_t)g.n[0] : (uint32_t)g.n[0] * (uint32_t)g.n[1];
            const int64_t in_inst = (axis == 1) ? (int64_t)outer * g.n[0] * g.n[1] + xt * LINES
                                                : (int64_t)outer * g.n[0] + xt * LINES;
            base = inst * g.M + in_inst;
            off0 = (uint32_t)l + (uint32_t)t * stride;
            dstep = (uint32_t)T * stride;
            jbase = in_inst + off0;
            jstride = stride;
        }
    }
    __device__ __forceinline__ uint32_t off(int m) const { return off0 + (uint32_t)m * dstep; }
    __device__ __forceinline__ int64_t j(int m) const { return jbase + (int64_t)((uint32_t)m * (uint32_t)FFTShape<N>::T * jstride); }
};

// Lattice indices of in-instance point j.
__device__ __forceinline__ void unflatten(const GroupDev& g, int64_t j, int& x, int& y, int& z) {
    x = (int)(j & (g.n[0] - 1));
    y = (int)((j >> g.log2n[0]) & (g.n[1] - 1));
    z = (int)(j >> (g.log2n[0] + g.log2n[1]));
}

template <int N, int MODE, bool CONTIG, int LINES>
__global__ void __launch_bounds__(FFTShape<N>::T* LINES) k_axis(GroupDev g, int axis, PassArgs args) {
    using F = FFTShape<N>;
    constexpr int R = F::R, T = F::T;
    constexpr int NF = (MODE == PASS_D1 || MODE == PASS_U) ? 1 : 2;
    using L = LdsLayout<N, LINES, CONTIG>;
    __shared__ c32 lds[NF * L::SIZE];
    const int t = CONTIG ? (int)(threadIdx.x % T) : (int)(threadIdx.x / LINES);
    const int l = CONTIG ? (int)(threadIdx.x / T) : (int)(threadIdx.x % LINES);
    const Tile<N, CONTIG, LINES> tile(g, axis, l, t);
    const float2* __restrict__ E = g.E[axis];
    const float2* __restrict__ tw = g.tw[axis];
    const int64_t o = g.offset + tile.base;
    float2* __restrict__ ps = args.psi ? args.psi + o : nullptr;
    float2* __restrict__ pa = args.A ? args.A + o : nullptr;
    float2* __restrict__ pb = args.B ? args.B + o : nullptr;
    const float2* __restrict__ x0 = args.aux0 ? args.aux0 + o : nullptr;
    const float2* __restrict__ x1 = args.aux1 ? args.aux1 + o : nullptr;
    double* __restrict__ vb = args.vbar ? args.vbar + o : nullptr;
    constexpr bool NEEDS_STEP = (MODE == PASS_FIRST || MODE == PASS_LAST1 || MODE == PASS_LAST2 ||
                                 MODE == PASS_U || MODE == PASS_AS);
    const int64_t step = NEEDS_STEP ? read_step(args.step_off, args.step_base) : 0;
    const uint32_t iid = g.id_base + (uint32_t)tile.inst;
    const float* __restrict__ Vg = g.Vgrid ? g.Vgrid + tile.inst * g.M : nullptr;

    // pointwise inputs of the right-hand side at element t + m T of this thread's line
    auto potential_at = [&](int m) {
        const int64_t j = tile.j(m);
        int x, y, z;
        unflatten(g, j, x, y, z);
        float V = trap_V(g, x, y, z);
        if (Vg) V += Vg[j];
        return V;
    };
    auto noise_at = [&](int m) {
        if (!g.has_noise) return make_float2(0.f, 0.f);
        const float2 zz = noise_z(g, tile.j(m), iid, step);
        return make_float2(g.noise_c * zz.x, g.noise_c * zz.y);
    };
    const c32 zero = make_float2(0.f, 0.f);

    c32 f[NF][R];
    if constexpr (MODE == PASS_D1 || MODE == PASS_FIRST) {
#pragma unroll
        for (int m = 0; m < R; m++) f[0][m] = tile.active ? ps[tile.off(m)] : zero;
        if constexpr (MODE == PASS_FIRST) {
#pragma unroll
            for (int m = 0; m < R; m++) f[1][m] = hG(g, f[0][m], potential_at(m), noise_at(m));
        }
    } else if constexpr (MODE == PASS_U) {
        // u = a + k3 from (a, k1)
#pragma unroll
        for (int m = 0; m < R; m++) {
            const c32 a = tile.active ? x0[tile.off(m)] : zero;
            const c32 k1 = tile.active ? x1[tile.off(m)] : zero;
            const float V = potential_at(m);
            const c32 nz = noise_at(m);
            const c32 k2 = hG(g, make_float2(fmaf(0.5f, k1.x, a.x), fmaf(0.5f, k1.y, a.y)), V, nz);
            const c32 k3 = hG(g, make_float2(fmaf(0.5f, k2.x, a.x), fmaf(0.5f, k2.y, a.y)), V, nz);
            f[0][m] = cadd(a, k3);
        }
    } else if constexpr (MODE == PASS_AW) {
        // adjoint of psi' = D acc + k4/6, k4 = h G(w): (lam, wbar = h J(w)^T lam/6)
#pragma unroll
        for (int m = 0; m < R; m++) {
            const c32 lam = tile.active ? ps[tile.off(m)] : zero;
            const c32 w = tile.active ? x0[tile.off(m)] : zero;
            const c32 k4b = cscale(lam, 1.0f / 6.0f);
            f[0][m] = lam;
            f[1][m] = hJT(g, w, potential_at(m), k4b);
            if (vb && tile.active) vb[tile.off(m)] += (double)hImconj(g, k4b, w);
        }
    } else {
#pragma unroll
        for (int m = 0; m < R; m++) {
            f[0][m] = tile.active ? pa[tile.off(m)] : zero;
            f[1][m] = tile.active ? pb[tile.off(m)] : zero;
        }
    }

    propagate<N, L, NF>(f, t, l, lds, tw, E, args.adj != 0);

    if (!tile.active) return;  // after the last barrier
    if constexpr (MODE == PASS_D1 || MODE == PASS_U) {
#pragma unroll
        for (int m = 0; m < R; m++) ps[tile.off(m)] = f[0][m];
    } else if constexpr (MODE == PASS_LAST1) {
#pragma unroll
        for (int m = 0; m < R; m++) {
            const float V = potential_at(m);
            const c32 nz = noise_at(m);
            const c32 a = f[0][m], k1 = f[1][m];
            const c32 k2 = hG(g, make_float2(fmaf(0.5f, k1.x, a.x), fmaf(0.5f, k1.y, a.y)), V, nz);
            const c32 k3 = hG(g, make_float2(fmaf(0.5f, k2.x, a.x), fmaf(0.5f, k2.y, a.y)), V, nz);
            const float sx = k1.x * (1.0f / 6.0f) + (k2.x + k3.x) * (1.0f / 3.0f);
            const float sy = k1.y * (1.0f / 6.0f) + (k2.y + k3.y) * (1.0f / 3.0f);
            pa[tile.off(m)] = cadd(a, k3);
            pb[tile.off(m)] = make_float2(a.x + sx, a.y + sy);
        }
    } else if constexpr (MODE == PASS_LAST2) {
#pragma unroll
        for (int m = 0; m < R; m++) {
            const c32 k4 = hG(g, f[0][m], potential_at(m), noise_at(m));
            ps[tile.off(m)] = make_float2(fmaf(k4.x, 1.0f / 6.0f, f[1][m].x), fmaf(k4.y, 1.0f / 6.0f, f[1][m].y));
        }
    } else if constexpr (MODE == PASS_AS) {
        // transposes of the stage combinations: (accbar, ubar) -> (abar, k1bar)
#pragma unroll
        for (int m = 0; m < R; m++) {
            const float V = potential_at(m);
            const c32 nz = noise_at(m);
            const c32 a = x0[tile.off(m)], k1 = x1[tile.off(m)];
            const c32 p2 = make_float2(fmaf(0.5f, k1.x, a.x), fmaf(0.5f, k1.y, a.y));
            const c32 k2 = hG(g, p2, V, nz);
            const c32 p3 = make_float2(fmaf(0.5f, k2.x, a.x), fmaf(0.5f, k2.y, a.y));
            const c32 accb = f[0][m], ub = f[1][m];
            const c32 k3b = make_float2(fmaf(accb.x, 1.0f / 3.0f, ub.x), fmaf(accb.y, 1.0f / 3.0f, ub.y));
            const c32 p3b = hJT(g, p3, V, k3b);
            const c32 k2b = make_float2(fmaf(accb.x, 1.0f / 3.0f, 0.5f * p3b.x), fmaf(accb.y, 1.0f / 3.0f, 0.5f * p3b.y));
            const c32 p2b = hJT(g, p2, V, k2b);
            const c32 k1b = make_float2(fmaf(accb.x, 1.0f / 6.0f, 0.5f * p2b.x), fmaf(accb.y, 1.0f / 6.0f, 0.5f * p2b.y));
            const c32 ab = make_float2(accb.x + ub.x + p3b.x + p2b.x, accb.y + ub.y + p3b.y + p2b.y);
            if (vb) vb[tile.off(m)] += (double)hImconj(g, k3b, p3) + (double)hImconj(g, k2b, p2);
            pa[tile.off(m)] = ab;
            pb[tile.off(m)] = k1b;
        }
    } else if constexpr (MODE == PASS_AF) {
        // psibar = D^T abar + h J(psi_n)^T (D^T k1bar)
#pragma unroll
        for (int m = 0; m < R; m++) {
            const c32 pn = x0[tile.off(m)];
            const c32 g0b = f[1][m];
            const c32 r = hJT(g, pn, potential_at(m), g0b);
            if (vb) vb[tile.off(m)] += (double)hImconj(g, g0b, pn);
            ps[tile.off(m)] = cadd(f[0][m], r);
        }
    } else {  // FIRST, D2, AW
#pragma unroll
        for (int m = 0; m < R; m++) {
            pa[tile.off(m)] = f[0][m];
            pb[tile.off(m)] = f[1][m];
        }
    }
}

// ---------------------------------------------------------------------------- 1D adjoint step

// Adjoint of one step of LPB whole lines: forward stages recomputed from psi_n in
// registers, then the two transposed D-pairs; lam (in/out) is the adjoint state and vbar
// accumulates the potential gradient.
template <int N, int LPB>
__global__ void __launch_bounds__(FFTShape<N>::T* LPB)
    k_line_adjoint(GroupDev g, const float2* __restrict__ psi_n, float2* __restrict__ lam, double* __restrict__ vbar,
                   int64_t step) {
    using F = FFTShape<N>;
    using L = LdsLayout<N, LPB, true>;
    constexpr int R = F::R, T = F::T;
    __shared__ c32 lds[2 * L::SIZE];
    const int t = threadIdx.x % T;
    const int l = threadIdx.x / T;
    const int64_t inst = (int64_t)blockIdx.x * LPB + l;
    const bool active = inst < g.batch;
    const int64_t base = g.offset + (active ? inst : 0) * N;
    const float2* __restrict__ E = g.E[0];
    const float2* __restrict__ tw = g.tw[0];
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
    // forward: (a, k1) = D (psi, hG(psi))
    c32 f[2][R];
#pragma unroll
    for (int m = 0; m < R; m++) {
        f[0][m] = active ? psi_n[base + t + m * T] : zero;
        f[1][m] = hG(g, f[0][m], V_at(m), nz_at(m));
    }
    propagate<N, L, 2>(f, t, l, lds, tw, E, false);
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
    propagate<N, L, 1>(w, t, l, lds, tw, E, false);
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
    propagate<N, L, 2>(b, t, l, lds, tw, E, true);
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
    propagate<N, L, 2>(b, t, l, lds, tw, E, true);
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

// ---------------------------------------------------------------------------- FP64 reductions

// Per line along `axis`: part[line][0] = sum_k k_a^2 |F_a psi|^2 / n_a, and on axis 0
// also part[line][1..3] = (sum |psi|^2, sum V |psi|^2, sum |psi|^4). Lines are numbered
// per instance (axis 0: by (z, y); strided: by (outer, x)), instances consecutive.
template <int N, bool CONTIG, int LINES>
__global__ void __launch_bounds__(FFTShape<N>::T* LINES)
    k_diag_axis(GroupDev g, int axis, const float2* __restrict__ psi, double kscale, double* __restrict__ part) {
    using F = FFTShape<N>;
    constexpr int R = F::R, T = F::T;
    using L = LdsLayout<N, LINES, CONTIG>;
    __shared__ c32 lds[L::SIZE];
    __shared__ double red[FFTShape<N>::T * LINES][4];
    const int t = CONTIG ? (int)(threadIdx.x % T) : (int)(threadIdx.x / LINES);
    const int l = CONTIG ? (int)(threadIdx.x / T) : (int)(threadIdx.x % LINES);
    const Tile<N, CONTIG, LINES> tile(g, axis, l, t);
    const float2* ps = psi + g.offset + tile.base;
    c32 f[1][R];
    double s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
    for (int m = 0; m < R; m++) {
        f[0][m] = tile.active ? ps[tile.off(m)] : make_float2(0.f, 0.f);
        if (axis == 0) {
            const int64_t j = tile.j(m);
            int x, y, z;
            unflatten(g, j, x, y, z);
            double V = (double)trap_V(g, x, y, z);
            if (g.Vgrid && tile.active) V += (double)g.Vgrid[tile.inst * g.M + j];
            const double m2 = (double)f[0][m].x * f[0][m].x + (double)f[0][m].y * f[0][m].y;
            s1 += m2;
            s2 += V * m2;
            s3 += m2 * m2;
        }
    }
    fft_line<N, -1, L, 1>(f, t, l, lds, g.tw[axis]);
    double s0 = 0.0;
#pragma unroll
    for (int m = 0; m < R; m++) {
        const int e = t + m * T;
        const int ks = e < N / 2 ? e : e - N;
        const double k = kscale * ks;
        const double a2 = (double)f[0][m].x * f[0][m].x + (double)f[0][m].y * f[0][m].y;
        s0 += k * k * a2;
    }
    // fixed-order reduction over the T threads of each line
    const int slot = l * T + t;
    red[slot][0] = s0;
    red[slot][1] = s1;
    red[slot][2] = s2;
    red[slot][3] = s3;
    __syncthreads();
    if (t == 0 && tile.active) {
        double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
        for (int i = 0; i < T; i++) {
            a0 += red[l * T + i][0];
            a1 += red[l * T + i][1];
            a2 += red[l * T + i][2];
            a3 += red[l * T + i][3];
        }
        // line number within the instance: (in-instance index of element 0) with the axis
        // coordinate removed
        const int64_t j0 = tile.jbase - (int64_t)t * tile.jstride;
        int64_t line;
        if (axis == 0) {
            line = j0 >> g.log2n[0];
        } else {
            int x, y, z;
            unflatten(g, j0, x, y, z);
            const int outer = (axis == 1) ? z : y;
            line = (int64_t)outer * g.n[0] + x;
        }
        line += tile.inst * (g.M >> g.log2n[axis]);
        double* o = part + line * 4;
        o[0] = a0 * (double)g.inv_n[axis];
        o[1] = a1;
        o[2] = a2;
        o[3] = a3;
    }
}

// One workgroup per instance: sums the line partials of every axis in a fixed order.
__global__ void __launch_bounds__(256)
    k_diag_final(GroupDev g, DiagConst c, const double* __restrict__ p0, const double* __restrict__ p1,
                 const double* __restrict__ p2, double* __restrict__ out, int* __restrict__ flag) {
    __shared__ double red[256][4];
    const int64_t inst = blockIdx.x;
    const int tid = threadIdx.x;
    double a[4] = {0, 0, 0, 0};
    const double* parts[3] = {p0, p1, p2};
    for (int ax = 0; ax < g.ndim; ax++) {
        const int64_t nl = g.M >> g.log2n[ax];
        const double* p = parts[ax] + inst * nl * 4;
        for (int64_t i = tid; i < nl; i += 256) {
            a[0] += p[i * 4 + 0];
            if (ax == 0) {
                a[1] += p[i * 4 + 1];
                a[2] += p[i * 4 + 2];
                a[3] += p[i * 4 + 3];
            }
        }
    }
    for (int q = 0; q < 4; q++) red[tid][q] = a[q];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s)
            for (int q = 0; q < 4; q++) red[tid][q] += red[tid + s][q];
        __syncthreads();
    }
    if (tid == 0) {
        const double N = c.dV * red[0][1];
        out[inst * 4 + 0] = N;
        out[inst * 4 + 1] = c.alpha * c.dV * red[0][0];
        out[inst * 4 + 2] = c.dV * red[0][2];
        out[inst * 4 + 3] = c.half_g * c.dV * red[0][3];
        if (!isfinite(N)) atomicOr(flag, 1);
    }
}

// Overlap c_b = dV sum conj(phi) psi_b: one workgroup per instance, fixed-order tree.
__global__ void __launch_bounds__(256)
    k_overlap(GroupDev g, double dV, const float2* __restrict__ phi, const float2* __restrict__ psi,
              double* __restrict__ out) {
    __shared__ double red[256][2];
    const int64_t inst = blockIdx.x;
    const int tid = threadIdx.x;
    const float2* p = psi + g.offset + inst * g.M;
    double re = 0.0, im = 0.0;
    for (int64_t j = tid; j < g.M; j += 256) {
        const double ar = phi[j].x, ai = phi[j].y, br = p[j].x, bi = p[j].y;
        re += ar * br + ai * bi;
        im += ar * bi - ai * br;
    }
    red[tid][0] = re;
    red[tid][1] = im;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) {
            red[tid][0] += red[tid + s][0];
            red[tid][1] += red[tid + s][1];
        }
        __syncthreads();
    }
    if (tid == 0) {
        out[inst * 2 + 0] = dV * red[0][0];
        out[inst * 2 + 1] = dV * red[0][1];
    }
}

// Per-point moments over the instances of a group (instance order fixed).
__global__ void k_moments(GroupDev g, const float2* __restrict__ psi, double* __restrict__ mean,
                          double* __restrict__ var) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= g.M) return;
    const float2* p = psi + g.offset + j;
    double s = 0.0;
    for (int64_t b = 0; b < g.batch; b++) {
        const float2 v = p[b * g.M];
        s += (double)v.x * v.x + (double)v.y * v.y;
    }
    const double mu = s / (double)g.batch;
    double ss = 0.0;
    for (int64_t b = 0; b < g.batch; b++) {
        const float2 v = p[b * g.M];
        const double d = (double)v.x * v.x + (double)v.y * v.y - mu;
        ss += d * d;
    }
    mean[j] = mu;
    var[j] = g.batch > 1 ? ss / (double)(g.batch - 1) : 0.0;
}

// ---------------------------------------------------------------------------- launchers

// LDS of a strided tile of w columns and nf fields must fit the 160 KiB of a CU.
constexpr bool fits_lds(int N, int w, int nf) { return (long)nf * N * w * 8 <= 128 * 1024; }

static int strided_lines(int N, int n0) {
    int w = N <= 256 ? 16 : (N == 512 ? 8 : 4);
    return w < n0 ? w : n0;
}

static int contig_lines(int N) {
    const int T = N < 16 ? 1 : N / 16;
    int l = 256 / T;
    return l < 1 ? 1 : l;
}

int axis_lines(int N, int axis, int n0) { return axis == 0 ? contig_lines(N) : strided_lines(N, n0); }

template <int N, int MODE, bool CONTIG, int LINES>
static hipError_t go_axis(const GroupDev& g, int axis, const PassArgs& a, hipStream_t s) {
    int64_t blocks;
    if (CONTIG)
        blocks = (g.batch * (g.M >> g.log2n[0]) + LINES - 1) / LINES;
    else
        blocks = g.batch * (g.M >> g.log2n[axis]) / LINES;
    hipLaunchKernelGGL((k_axis<N, MODE, CONTIG, LINES>), dim3((unsigned)blocks), dim3(FFTShape<N>::T * LINES), 0, s,
                       g, axis, a);
    return hipGetLastError();
}

// passes that run only on axis 0 / only on the last (strided) axis
constexpr bool contig_only(int mode) { return mode == PASS_FIRST || mode == PASS_U || mode == PASS_AW; }
constexpr bool strided_only(int mode) {
    return mode == PASS_LAST1 || mode == PASS_LAST2 || mode == PASS_AS || mode == PASS_AF;
}

template <int N, int MODE>
static hipError_t go_axis_n(const GroupDev& g, int axis, const PassArgs& a, hipStream_t s) {
    constexpr int T = FFTShape<N>::T;
    constexpr int CL = (256 / T) < 1 ? 1 : 256 / T;
    if (axis == 0) {
        if constexpr (strided_only(MODE)) {
            return hipErrorInvalidValue;
        } else {
            return go_axis<N, MODE, true, CL>(g, axis, a, s);
        }
    }
    if constexpr (contig_only(MODE)) {
        return hipErrorInvalidValue;
    } else {
        const int w = strided_lines(N, g.n[0]);
        switch (w) {
            case 16:
                if constexpr (T * 16 <= 1024 && fits_lds(N, 16, 2)) return go_axis<N, MODE, false, 16>(g, axis, a, s);
                break;
            case 8:
                if constexpr (T * 8 <= 1024 && fits_lds(N, 8, 2)) return go_axis<N, MODE, false, 8>(g, axis, a, s);
                break;
            case 4: return go_axis<N, MODE, false, 4>(g, axis, a, s);
            default: break;
        }
        return hipErrorInvalidValue;
    }
}

template <int MODE>
static hipError_t go_axis_mode(const GroupDev& g, int axis, const PassArgs& a, hipStream_t s) {
    switch (g.n[axis]) {
        case 8: return go_axis_n<8, MODE>(g, axis, a, s);
        case 16: return go_axis_n<16, MODE>(g, axis, a, s);
        case 32: return go_axis_n<32, MODE>(g, axis, a, s);
        case 64: return go_axis_n<64, MODE>(g, axis, a, s);
        case 128: return go_axis_n<128, MODE>(g, axis, a, s);
        case 256: return go_axis_n<256, MODE>(g, axis, a, s);
        case 512: return go_axis_n<512, MODE>(g, axis, a, s);
        case 1024: return go_axis_n<1024, MODE>(g, axis, a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_axis(const GroupDev& g, int axis, int mode, const PassArgs& a, hipStream_t s) {
    switch (mode) {
        case PASS_D1: return go_axis_mode<PASS_D1>(g, axis, a, s);
        case PASS_D2: return go_axis_mode<PASS_D2>(g, axis, a, s);
        case PASS_FIRST: return go_axis_mode<PASS_FIRST>(g, axis, a, s);
        case PASS_LAST1: return go_axis_mode<PASS_LAST1>(g, axis, a, s);
        case PASS_LAST2: return go_axis_mode<PASS_LAST2>(g, axis, a, s);
        case PASS_U: return go_axis_mode<PASS_U>(g, axis, a, s);
        case PASS_AW: return go_axis_mode<PASS_AW>(g, axis, a, s);
        case PASS_AS: return go_axis_mode<PASS_AS>(g, axis, a, s);
        case PASS_AF: return go_axis_mode<PASS_AF>(g, axis, a, s);
        default: return hipErrorInvalidValue;
    }
}

template <int N>
static hipError_t go_line_adj(const GroupDev& g, const float2* psi_n, float2* lam, double* vbar, int64_t step,
                              hipStream_t s) {
    constexpr int T = FFTShape<N>::T;
    constexpr int LPB = T >= 64 ? 1 : 64 / T;
    const int64_t blocks = (g.batch + LPB - 1) / LPB;
    hipLaunchKernelGGL((k_line_adjoint<N, LPB>), dim3((unsigned)blocks), dim3(T * LPB), 0, s, g, psi_n, lam, vbar,
                       step);
    return hipGetLastError();
}

hipError_t launch_line_adjoint(const GroupDev& g, const float2* psi_n, float2* lam, double* vbar, int64_t step,
                               hipStream_t s) {
    switch (g.n[0]) {
        case 8: return go_line_adj<8>(g, psi_n, lam, vbar, step, s);
        case 16: return go_line_adj<16>(g, psi_n, lam, vbar, step, s);
        case 32: return go_line_adj<32>(g, psi_n, lam, vbar, step, s);
        case 64: return go_line_adj<64>(g, psi_n, lam, vbar, step, s);
        case 128: return go_line_adj<128>(g, psi_n, lam, vbar, step, s);
        case 256: return go_line_adj<256>(g, psi_n, lam, vbar, step, s);
        case 512: return go_line_adj<512>(g, psi_n, lam, vbar, step, s);
        case 1024: return go_line_adj<1024>(g, psi_n, lam, vbar, step, s);
        case 2048: return go_line_adj<2048>(g, psi_n, lam, vbar, step, s);
        case 4096: return go_line_adj<4096>(g, psi_n, lam, vbar, step, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_vbar_to_float(const double* vbar, float* out, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_vbar_to_float, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, vbar, out, n);
    return hipGetLastError();
}

template <int N>
static hipError_t go_line(const GroupDev& g, float2* psi, int nsteps, int64_t step_off, const int64_t* step_base,
                          hipStream_t s) {
    constexpr int T = FFTShape<N>::T;
    constexpr int LPB = T >= 64 ? 1 : 64 / T;
    const int64_t blocks = (g.batch + LPB - 1) / LPB;
    hipLaunchKernelGGL((k_line_step<N, LPB>), dim3((unsigned)blocks), dim3(T * LPB), 0, s, g, psi, nsteps, step_off,
                       step_base);
    return hipGetLastError();
}

hipError_t launch_line_step(const GroupDev& g, float2* psi, int nsteps, int64_t step_off, const int64_t* step_base,
                            hipStream_t s) {
    switch (g.n[0]) {
        case 8: return go_line<8>(g, psi, nsteps, step_off, step_base, s);
        case 16: return go_line<16>(g, psi, nsteps, step_off, step_base, s);
        case 32: return go_line<32>(g, psi, nsteps, step_off, step_base, s);
        case 64: return go_line<64>(g, psi, nsteps, step_off, step_base, s);
        case 128: return go_line<128>(g, psi, nsteps, step_off, step_base, s);
        case 256: return go_line<256>(g, psi, nsteps, step_off, step_base, s);
        case 512: return go_line<512>(g, psi, nsteps, step_off, step_base, s);
        case 1024: return go_line<1024>(g, psi, nsteps, step_off, step_base, s);
        case 2048: return go_line<2048>(g, psi, nsteps, step_off, step_base, s);
        case 4096: return go_line<4096>(g, psi, nsteps, step_off, step_base, s);
        default: return hipErrorInvalidValue;
    }
}

template <int N, bool CONTIG, int LINES>
static hipError_t go_diag(const GroupDev& g, int axis, const float2* psi, double kscale, double* part,
                          hipStream_t s) {
    int64_t blocks;
    if (CONTIG)
        blocks = (g.batch * (g.M >> g.log2n[0]) + LINES - 1) / LINES;
    else
        blocks = g.batch * (g.M >> g.log2n[axis]) / LINES;
    hipLaunchKernelGGL((k_diag_axis<N, CONTIG, LINES>), dim3((unsigned)blocks), dim3(FFTShape<N>::T * LINES), 0, s,
                       g, axis, psi, kscale, part);
    return hipGetLastError();
}

template <int N>
static hipError_t go_diag_n(const GroupDev& g, int axis, const float2* psi, double kscale, double* part,
                            hipStream_t s) {
    constexpr int T = FFTShape<N>::T;
    constexpr int CL = (256 / T) < 1 ? 1 : 256 / T;
    if (axis == 0) return go_diag<N, true, CL>(g, axis, psi, kscale, part, s);
    const int w = strided_lines(N, g.n[0]);
    switch (w) {
        case 16:
            if constexpr (T * 16 <= 1024 && fits_lds(N, 16, 1))
                return go_diag<N, false, 16>(g, axis, psi, kscale, part, s);
            break;
        case 8:
            if constexpr (T * 8 <= 1024 && fits_lds(N, 8, 1)) return go_diag<N, false, 8>(g, axis, psi, kscale, part, s);
            break;
        case 4: return go_diag<N, false, 4>(g, axis, psi, kscale, part, s);
        default: break;
    }
    return hipErrorInvalidValue;
}

hipError_t launch_diag_axis(const GroupDev& g, int axis, const float2* psi, double kscale, double* part,
                            hipStream_t s) {
    switch (g.n[axis]) {
        case 8: return go_diag_n<8>(g, axis, psi, kscale, part, s);
        case 16: return go_diag_n<16>(g, axis, psi, kscale, part, s);
        case 32: return go_diag_n<32>(g, axis, psi, kscale, part, s);
        case 64: return go_diag_n<64>(g, axis, psi, kscale, part, s);
        case 128: return go_diag_n<128>(g, axis, psi, kscale, part, s);
        case 256: return go_diag_n<256>(g, axis, psi, kscale, part, s);
        case 512: return go_diag_n<512>(g, axis, psi, kscale, part, s);
        case 1024: return go_diag_n<1024>(g, axis, psi, kscale, part, s);
        case 2048:
            if (axis == 0) return go_diag<2048, true, 1>(g, axis, psi, kscale, part, s);
            return hipErrorInvalidValue;
        case 4096:
            if (axis == 0) return go_diag<4096, true, 1>(g, axis, psi, kscale, part, s);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_diag_final(const GroupDev& g, const DiagConst& c, const double* p0, const double* p1,
                             const double* p2, double* out, int* flag, hipStream_t s) {
    hipLaunchKernelGGL(k_diag_final, dim3((unsigned)g.batch), dim3(256), 0, s, g, c, p0, p1, p2, out, flag);
    return hipGetLastError();
}

hipError_t launch_overlap(const GroupDev& g, double dV, const float2* phi, const float2* psi, double* out,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_overlap, dim3((unsigned)g.batch), dim3(256), 0, s, g, dV, phi, psi, out);
    return hipGetLastError();
}

hipError_t launch_moments(const GroupDev& g, const float2* psi, double* mean, double* var, hipStream_t s) {
    const int64_t blocks = (g.M + 255) / 256;
    hipLaunchKernelGGL(k_moments, dim3((unsigned)blocks), dim3(256), 0, s, g, psi, mean, var);
    return hipGetLastError();
}

hipError_t launch_counter(int64_t* c, int64_t v, int add, hipStream_t s) {
    hipLaunchKernelGGL(k_counter, dim3(1), dim3(64), 0, s, c, v, add);
    return hipGetLastError();
}

hipError_t launch_philox(uint32_t k0, uint32_t k1, const uint32_t* ctr, int64_t n, uint32_t* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_philox, dim3((unsigned)blocks), dim3(256), 0, s, k0, k1, (const uint4*)ctr, n, (uint4*)out);
    return hipGetLastError();
}

hipError_t launch_noise(const GroupDev& g, int64_t step, float2* xi, hipStream_t s) {
    const int64_t n = g.batch * g.M;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_noise, dim3((unsigned)blocks), dim3(256), 0, s, g, step, xi);
    return hipGetLastError();
}

template <int N>
static hipError_t go_fft(const float2* in, float2* out, int64_t nlines, int sign, const float2* tw, hipStream_t s) {
    constexpr int T = FFTShape<N>::T;
    constexpr int LINES = T >= 256 ? 1 : 256 / T;
    const int64_t blocks = (nlines + LINES - 1) / LINES;
    hipLaunchKernelGGL((k_fft_lines<N, LINES>), dim3((unsigned)blocks), dim3(T * LINES), 0, s, in, out, nlines, sign,
                       tw);
    return hipGetLastError();
}

hipError_t launch_fft_lines(const float2* in, float2* out, int64_t n, int64_t nlines, int sign, const float2* tw,
                            hipStream_t s) {
    switch (n) {
        case 8: return go_fft<8>(in, out, nlines, sign, tw, s);
        case 16: return go_fft<16>(in, out, nlines, sign, tw, s);
        case 32: return go_fft<32>(in, out, nlines, sign, tw, s);
        case 64: return go_fft<64>(in, out, nlines, sign, tw, s);
        case 128: return go_fft<128>(in, out, nlines, sign, tw, s);
        case 256: return go_fft<256>(in, out, nlines, sign, tw, s);
        case 512: return go_fft<512>(in, out, nlines, sign, tw, s);
        case 1024: return go_fft<1024>(in, out, nlines, sign, tw, s);
        case 2048: return go_fft<2048>(in, out, nlines, sign, tw, s);
        case 4096: return go_fft<4096>(in, out, nlines, sign, tw, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace rk4ip
