// pass_common.h -- the per-axis pass kernel of the RK4IP step, its tile mapping and the
// launch templates shared by the forward and adjoint kernel files.
//
// The step (Dennis, Hope & Johnsson, arXiv:1204.4255: classic RK4, Sec. 3.5, in the
// interaction picture of Sec. 3.6 with the picture origin at the step midpoint) is
//   a  = D psi,   k1 = D[h G(psi)],   k2 = h G(a + k1/2),   k3 = h G(a + k2/2),
//   k4 = h G(D(a + k3)),   psi' = D(a + k1/6 + k2/3 + k3/3) + k4/6,
// with D = e^{L h/2} applied per lattice axis (Sec. 3.2 factorisation): FFT along the
// axis, multiply by e^{L_a h/2}, inverse FFT. The four D applications come in two pairs
// of two fields. D commutes across axes, so the second pair can sweep the axes in the
// reverse order of the first; then the two passes on the last axis and the two on axis 0
// (the end of one step and the start of the next) each fuse into one pass. On a 2D/3D
// lattice every pass reads and writes two complex64 fields once:
//   FIRST (axis 0):  psi    -> (psi, hG(psi)) -> D_0 -> (A, B)         opens a run of steps
//   D2    (middle):  (A, B) -> D_a -> (A, B)
//   LF    (last):    (A, B) -> D_a -> (a, k1); k2, k3; u = a + k3,
//                              acc = a + k1/6 + k2/3 + k3/3 -> D_a -> (A, B)
//   D2    (middle, second sweep)
//   XF    (axis 0):  (A, B) -> D_0 -> psi' = D acc + hG(D u)/6; (psi', hG(psi')) -> D_0 -> (A, B)
//   LAST2 (axis 0):  (A, B) -> D_0 -> psi' -> psi                      closes the run
// The noise of a step is drawn wherever that step evaluates G (XF draws step n-1's for k4
// and step n's for the next start).
//
// The semi-implicit step (Sec. 3.5, in the same midpoint picture: a = D psi, m = a +
// (h/2) G(m) by three fixed-point iterations, psi' = D(2m - a)) works on psi in place:
//   D1 (axis 0, half step, opens a run); D1 (middle axes);
//   SI (last axis): psi -> D_a -> a; m; 2m - a -> D_a -> psi;  D1 (middle axes);
//   D1 (axis 0) twice in registers where two steps meet (the same arithmetic as closing
//   one run and opening the next, so split runs stay bitwise equal), or once to close.
// A 1D line fits one workgroup, so the whole step (eight transforms) runs in registers
// and LDS with one read and one write of psi (k_line_step), optionally for several
// steps per launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "device_common.h"
#include "launch.h"

namespace rk4ip {

__device__ __forceinline__ int64_t read_step(int64_t step_off, const int64_t* step_base) {
    return step_off + (step_base ? *step_base : 0);
}

// Stage an axis's twiddles (in the transform's stage-major order) and its (E - 1)/n
// table into LDS (the caller synchronises).
template <class F, class V>
__device__ __forceinline__ void stage_tables(V* s_tw, V* s_E, const V* __restrict__ tw, const V* __restrict__ E) {
    stage_twiddles<F>(s_tw, tw);
    if (s_E) {
        for (int i = threadIdx.x; i < F::NN; i += blockDim.x) s_E[i] = E[i];
    }
}

// D_a on NF lines held in registers, in delta form: f <- f + F^{-1}[(E_a - 1)/n F f]
// (adj: the transpose, with the conjugate multiplier). tw and E point to LDS copies of
// the tables. V is the working type of the transform: float2, or double2 for the
// FP64-transform form (the correction is formed and added to f in FP64 and rounded to
// FP32 once). All threads of the block call it.
__device__ __forceinline__ c32 widen(c32 a, c32) { return a; }
__device__ __forceinline__ c64 widen(c32 a, c64) { return make_double2((double)a.x, (double)a.y); }
__device__ __forceinline__ c32 narrow(c32 a) { return a; }
__device__ __forceinline__ c32 narrow(c64 a) { return make_float2((float)a.x, (float)a.y); }

template <class F, class L, int NF, class V>
__device__ __forceinline__ void propagate(c32 (&f)[NF][F::R], int t, int l, V* lds, const V* tw, const V* E,
                                          bool adj) {
    V d[NF][F::R];
#pragma unroll
    for (int q = 0; q < NF; q++)
#pragma unroll
        for (int m = 0; m < F::R; m++) d[q][m] = widen(f[q][m], V{});
    fft_line<F, -1, L, NF>(d, t, l, lds, tw);
#pragma unroll
    for (int m = 0; m < F::R; m++) {
        V cs = E[t + m * F::T];
        if (adj) cs.y = -cs.y;
#pragma unroll
        for (int q = 0; q < NF; q++) d[q][m] = cmul(d[q][m], cs);
    }
    fft_line<F, +1, L, NF>(d, t, l, lds, tw);
#pragma unroll
    for (int q = 0; q < NF; q++)
#pragma unroll
        for (int m = 0; m < F::R; m++) f[q][m] = narrow(cadd(widen(f[q][m], V{}), d[q][m]));
}

// The non-local potential of a line (1D groups): V_c = F^{-1}[kh F|f|^2] with kh the
// kernel's transform times dV/n, so V_c(x_i) = dV sum_j K(x_i - x_j) |f_j|^2 on the
// periodic line. W: the transform's working type.
template <class F, class L, class W>
__device__ __forceinline__ void conv_V(const c32 (&f)[F::R], float (&vc)[F::R], int t, int l, W* lds, const W* tw,
                                       const float2* __restrict__ kh) {
    constexpr int R = F::R, T = F::T;
    W d[1][R];
#pragma unroll
    for (int m = 0; m < R; m++) d[0][m] = widen(make_float2(fmaf(f[m].x, f[m].x, f[m].y * f[m].y), 0.f), W{});
    fft_line<F, -1, L, 1>(d, t, l, lds, tw);
#pragma unroll
    for (int m = 0; m < R; m++) d[0][m] = cmul(d[0][m], widen(kh[t + m * T], W{}));
    fft_line<F, +1, L, 1>(d, t, l, lds, tw);
#pragma unroll
    for (int m = 0; m < R; m++) vc[m] = (float)d[0][m].x;
}

// Which lines a workgroup owns and where element e of its line l lives.
// CONTIG: LINES consecutive lines along axis 0 (threads of a line are adjacent lanes).
// strided: LINES adjacent x columns of one (instance, outer index) along axis 1 or 2
// (adjacent lanes hold adjacent columns, so each row segment is one coalesced access).
// Addresses are a workgroup-uniform 64-bit tile base plus 32-bit per-thread offsets,
// shared by every field the pass touches.
// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2. Give every
// XCD a contiguous run of tiles instead, so that neighbouring strided tiles (which share
// 128-byte lines when a tile row is narrower than a line) run on the same L2 at about the
// same time. A bijection of [0, G).
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t G) {
    const uint32_t q = G >> 3, r = G & 7u, x = b & 7u;
    return x * q + (x < r ? x : r) + (b >> 3);
}

template <class F, bool CONTIG, int LINES>
struct Tile {
    static constexpr int N = F::NN;
    int64_t base;      // uniform: group-relative point index of the tile origin
    uint32_t off0;     // this thread's element 0 relative to base
    uint32_t dstep;    // offset between element t + m T and t + (m+1) T
    int64_t inst;      // instance of this thread's line
    int64_t jbase;     // in-instance index of this thread's element 0 (noise counter, Vgrid)
    uint32_t jstride;  // in-instance index step per element along the axis
    bool active;

    // bid: this workgroup's tile among the nblk tiles of the group's pass
    __device__ __forceinline__ Tile(const GroupDev& g, int axis, int l, int t, uint32_t bid, uint32_t nblk) {
        constexpr int T = F::T;
        // every count below is a power of two: shifts and masks, no division
        if constexpr (CONTIG) {
            const int lpi = g.log2n[1] + g.log2n[2];  // log2 of the lines per instance
            const int64_t nlines = g.batch << lpi;
            const int64_t line = (int64_t)bid * LINES + l;
            active = line < nlines;
            const int64_t ln = active ? line : 0;
            base = (int64_t)bid * LINES * N;
            off0 = (uint32_t)(l * N + t);
            dstep = T;
            inst = ln >> lpi;
            jbase = (ln & ((int64_t(1) << lpi) - 1)) * N + t;
            jstride = 1;
        } else {
            const int xt_log = g.log2n[0] - ilog2(LINES);  // column tiles per row
            const int outer_log = (axis == 1) ? g.log2n[2] : g.log2n[1];
            // tiles whose rows are narrower than a 128-byte line share lines with a neighbour
            bid = (LINES * 8 < 128) ? xcd_tile(bid, nblk) : bid;
            const int xt = (int)(bid & ((1u << xt_log) - 1u));
            bid >>= xt_log;
            const int outer = (int)(bid & ((1u << outer_log) - 1u));
            inst = (int64_t)(bid >> outer_log);
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
    // byte offset of element t + m T for a field of float2 (the tile spans < 4 GiB)
    __device__ __forceinline__ uint32_t b8(int m) const { return (off0 + (uint32_t)m * dstep) * 8u; }
    __device__ __forceinline__ int64_t j(int m) const { return jbase + (int64_t)((uint32_t)m * (uint32_t)F::T * jstride); }
};

// Access at a 32-bit byte offset from a workgroup-uniform base: lets the compiler use the
// scalar-base form of the global load/store instead of a 64-bit address per element.
__device__ __forceinline__ float2 ld2(const float2* base, uint32_t boff) {
    return *reinterpret_cast<const float2*>(reinterpret_cast<const char*>(base) + boff);
}
__device__ __forceinline__ void st2(float2* base, uint32_t boff, float2 v) {
    *reinterpret_cast<float2*>(reinterpret_cast<char*>(base) + boff) = v;
}
__device__ __forceinline__ double ldd(const double* base, uint32_t boff) {
    return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(base) + boff);
}
__device__ __forceinline__ void std_(double* base, uint32_t boff, double v) {
    *reinterpret_cast<double*>(reinterpret_cast<char*>(base) + boff) = v;
}

// Lattice indices of in-instance point j.
__device__ __forceinline__ void unflatten(const GroupDev& g, int64_t j, int& x, int& y, int& z) {
    x = (int)(j & (g.n[0] - 1));
    y = (int)((j >> g.log2n[0]) & (g.n[1] - 1));
    z = (int)(j >> (g.log2n[0] + g.log2n[1]));
}

constexpr int fields_of(int mode) { return (mode == PASS_D1 || mode == PASS_SI) ? 1 : 2; }

// The fused adjoint passes (own bodies below).
constexpr bool adj_fused(int mode) { return mode == PASS_D2U || mode == PASS_XAW; }

// passes whose pointwise work evaluates G (and so may draw noise)
constexpr bool uses_rhs(int mode) {
    return mode == PASS_FIRST || mode == PASS_LAST2 || mode == PASS_AS ||
           mode == PASS_LF || mode == PASS_XF || mode == PASS_SI || mode == PASS_D2U;
}

// SEQ = 0: both fields go through the transform together (one exchange buffer each).
// SEQ = 1: they share one buffer and go through one after the other (half the LDS, a
//          lower register peak, twice the barriers).
// SEQ = 2: as 1, and the second field is only loaded once the first is transformed
//          (lowest register peak, fewer loads in flight per wave).
// SEQ = 3: one thread per field: the workgroup has twice the threads, its first half
//          carries field 0 and its second half field 1 of the same lines, each through its
//          own exchange buffer; where a pass combines the two fields pointwise, the halves
//          swap values through LDS. Twice the threads per line for lattices with few lines,
//          and half the registers per thread (forward passes with two fields, radix 8).
// RR: values per thread in the transform (16, or 8 for half the registers and one more
// LDS exchange per transform).
// OCC: the minimum waves per SIMD the register allocation must allow (1 = no constraint;
// 4 is a tuned variant for the radix-8 passes, whose allocation otherwise lands just
// above the 128 VGPRs that four waves need).
// LDS of one workgroup of the pass: the exchange buffers, then the twiddles and the
// propagator table (V entries).
template <int N, int MODE, bool CONTIG, int LINES, int SEQ, int RR, bool P64>
struct AxisLds {
    using V = typename std::conditional<P64, c64, c32>::type;
    using L = LdsLayout<N, LINES, CONTIG, FFTShape<N, RR>::R>;
    static constexpr int BUF = ((SEQ == 1 || SEQ == 2) ? 1 : fields_of(MODE)) * L::SIZE;
    static constexpr int ENTRIES = BUF + 2 * N;
    static constexpr size_t BYTES = sizeof(V) * (size_t)ENTRIES;
};

// The pass on tile `bid` of the `nblk` tiles of group g (one workgroup of T x LINES
// threads); smem holds AxisLds<...>::ENTRIES values of the working type.
template <int N, int MODE, bool CONTIG, int LINES, bool NOISE, int SEQ, int RR, bool P64>
__device__ __forceinline__ void axis_body(const GroupDev& g, int axis, const PassArgs& args, uint32_t bid, uint32_t nblk,
                                          typename AxisLds<N, MODE, CONTIG, LINES, SEQ, RR, P64>::V* smem) {
    using F = FFTShape<N, RR>;
    using V = typename std::conditional<P64, c64, c32>::type;  // transform working type
    constexpr int R = F::R, T = F::T;
    constexpr int NF = fields_of(MODE);
    using L = LdsLayout<N, LINES, CONTIG, R>;
    using A = AxisLds<N, MODE, CONTIG, LINES, SEQ, RR, P64>;
    V* lds = smem;
    V* tw = smem + A::BUF;
    V* E = tw + N;
    if constexpr (P64)
        stage_tables<F>(tw, E, g.tw64[axis], g.E64[axis]);
    else
        stage_tables<F>(tw, E, g.tw[axis], g.E[axis]);
    const int t = CONTIG ? (int)(threadIdx.x % T) : (int)(threadIdx.x / LINES);
    const int l = CONTIG ? (int)(threadIdx.x / T) : (int)(threadIdx.x % LINES);
    const Tile<F, CONTIG, LINES> tile(g, axis, l, t, bid, nblk);
    const int64_t o = g.offset + tile.base;
    float2* __restrict__ ps = args.psi ? args.psi + o : nullptr;
    float2* __restrict__ pa = args.A ? args.A + o : nullptr;
    float2* __restrict__ pb = args.B ? args.B + o : nullptr;
    const float2* __restrict__ x0 = args.aux0 ? args.aux0 + o : nullptr;
    const float2* __restrict__ x1 = args.aux1 ? args.aux1 + o : nullptr;
    double* __restrict__ vb = args.vbar ? args.vbar + o : nullptr;
    constexpr bool NEEDS_STEP = uses_rhs(MODE);
    const int64_t step = NEEDS_STEP ? read_step(args.step_off, args.step_base) : 0;
    const uint32_t iid = g.id_base + (uint32_t)tile.inst;
    const float* __restrict__ Vg = g.Vgrid ? g.Vgrid + tile.inst * g.M : nullptr;

    // The trap potential along the line: the other axes' part once per thread, the
    // axis's own term per element.
    float V_other = 0.0f;
    {
        int x, y, z;
        unflatten(g, tile.j(0), x, y, z);
        const int c[3] = {x, y, z};
#pragma unroll
        for (int a = 0; a < 3; a++) {
            if (a == axis || a >= g.ndim) continue;
            const float xa = fmaf((float)c[a], g.dx[a], g.lo[a]);
            V_other = fmaf(g.half_trap[a] * xa, xa, V_other);
        }
    }
    const float ht_axis = g.half_trap[axis], lo_axis = g.lo[axis], dx_axis = g.dx[axis];
    auto potential_at = [&](int m) {
        const float xa = fmaf((float)(t + m * T), dx_axis, lo_axis);
        float V = fmaf(ht_axis * xa, xa, V_other);
        if (Vg) V += Vg[tile.j(m)];
        return V;
    };
    auto noise_at = [&](int m, int64_t st) {
        if constexpr (!NOISE) {
            return make_float2(0.f, 0.f);
        } else {
            const float2 zz = noise_z(g, tile.j(m), iid, st);
            return make_float2(g.noise_c * zz.x, g.noise_c * zz.y);
        }
    };
    // the potential G sees at step st: V plus the real Wiener noise in the potential
    auto pot_at = [&](int m, int64_t st) {
        float V = potential_at(m);
        if constexpr (NOISE) {
            if (g.has_vnoise) V += vnoise(g, tile.j(m), iid, st);  // uniform
        }
        return V;
    };
    const c32 zero = make_float2(0.f, 0.f);

    // RK4 stages at the midpoint picture: (a, k1) -> (u, acc) in place
    auto stages = [&](c32& f0, c32& f1, float V, c32 nz) {
        const c32 a = f0, k1 = f1;
        const c32 k2 = hG(g, make_float2(fmaf(0.5f, k1.x, a.x), fmaf(0.5f, k1.y, a.y)), V, nz);
        const c32 k3 = hG(g, make_float2(fmaf(0.5f, k2.x, a.x), fmaf(0.5f, k2.y, a.y)), V, nz);
        const float sx = k1.x * (1.0f / 6.0f) + (k2.x + k3.x) * (1.0f / 3.0f);
        const float sy = k1.y * (1.0f / 6.0f) + (k2.y + k3.y) * (1.0f / 3.0f);
        f0 = cadd(a, k3);
        f1 = make_float2(a.x + sx, a.y + sy);
    };

    c32 f[NF][R];
    if constexpr (MODE == PASS_D1 || MODE == PASS_FIRST || MODE == PASS_SI) {
#pragma unroll
        for (int m = 0; m < R; m++) f[0][m] = tile.active ? ld2(ps, tile.b8(m)) : zero;
        if constexpr (MODE == PASS_FIRST) {
#pragma unroll
            for (int m = 0; m < R; m++) f[1][m] = hG(g, f[0][m], pot_at(m, step), noise_at(m, step));
        }
    } else {
#pragma unroll
        for (int m = 0; m < R; m++) f[0][m] = tile.active ? ld2(pa, tile.b8(m)) : zero;
        if constexpr (SEQ != 2) {
#pragma unroll
            for (int m = 0; m < R; m++) f[1][m] = tile.active ? ld2(pb, tile.b8(m)) : zero;
        }
    }

    // D_axis on the registers (the first time in a pass, the second field may still have
    // to be loaded: SEQ == 2)
    auto transform = [&](bool first) {
        if constexpr (SEQ != 0 && NF == 2) {
            c32(&f0)[1][R] = *reinterpret_cast<c32(*)[1][R]>(&f[0]);
            c32(&f1)[1][R] = *reinterpret_cast<c32(*)[1][R]>(&f[1]);
            propagate<F, L, 1>(f0, t, l, lds, tw, E, args.adj != 0);
            if constexpr (SEQ == 2) {
                if (first) {
#pragma unroll
                    for (int m = 0; m < R; m++) f[1][m] = tile.active ? ld2(pb, tile.b8(m)) : zero;
                }
            }
            propagate<F, L, 1>(f1, t, l, lds, tw, E, args.adj != 0);
        } else {
            propagate<F, L, NF>(f, t, l, lds, tw, E, args.adj != 0);
        }
    };

    __syncthreads();  // tables staged (the loads above overlap the copy)
    transform(true);
    if constexpr (MODE == PASS_D1) {
        if (args.twice) transform(false);  // uniform over the grid
    }

    if constexpr (MODE == PASS_AS) {
        // transposes of the stage combinations: (accbar, ubar) -> (abar, k1bar), then the
        // transposed propagator of this axis on both (the pass runs on the last axis, whose
        // share of D^T (abar, k1bar) is applied here rather than in a pass of its own)
#pragma unroll
        for (int m = 0; m < R; m++) {
            const float V = potential_at(m);
            const c32 nz = noise_at(m, step);
            const c32 a = ld2(x0, tile.b8(m)), k1 = ld2(x1, tile.b8(m));
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
            if (vb) std_(vb, tile.b8(m), ldd(vb, tile.b8(m)) + (double)hImconj(g, k3b, p3) + (double)hImconj(g, k2b, p2));
            f[0][m] = ab;
            f[1][m] = k1b;
        }
        transform(false);
    }

    if constexpr (MODE == PASS_LF || MODE == PASS_XF || MODE == PASS_SI) {
        // the work between the two transforms of a fused pass (every thread takes part in
        // the second transform's barriers, active or not)
#pragma unroll
        for (int m = 0; m < R; m++) {
            const float V = pot_at(m, step);
            if constexpr (MODE == PASS_SI) {
                // semi-implicit step at the midpoint picture: m = a + (h/2) G(m) by three
                // fixed-point iterations from m = a, then the end of the step 2m - a
                const c32 a = f[0][m], nz = noise_at(m, step);
                c32 mid = a;
#pragma unroll
                for (int it = 0; it < 3; it++) {
                    const c32 k = hG(g, mid, V, nz);
                    mid = make_float2(fmaf(0.5f, k.x, a.x), fmaf(0.5f, k.y, a.y));
                }
                f[0][m] = make_float2(fmaf(2.0f, mid.x, -a.x), fmaf(2.0f, mid.y, -a.y));
            } else if constexpr (MODE == PASS_LF) {
                stages(f[0][m], f[1][m], V, noise_at(m, step));
            } else {
                // end of step n-1: psi_n = D acc + hG(D u)/6, then the start of step n:
                // (psi_n, h G(psi_n))
                const c32 k4 = hG(g, f[0][m], pot_at(m, step - 1), noise_at(m, step - 1));
                const c32 psi_n = make_float2(fmaf(k4.x, 1.0f / 6.0f, f[1][m].x), fmaf(k4.y, 1.0f / 6.0f, f[1][m].y));
                f[0][m] = psi_n;
                f[1][m] = hG(g, psi_n, V, noise_at(m, step));
            }
        }
        transform(false);
    }

    if (!tile.active) return;  // after the last barrier
    if constexpr (MODE == PASS_D1 || MODE == PASS_SI) {
#pragma unroll
        for (int m = 0; m < R; m++) st2(ps, tile.b8(m), f[0][m]);
    } else if constexpr (MODE == PASS_LAST2) {
        float2* __restrict__ po = args.psi_out ? args.psi_out + o : ps;
#pragma unroll
        for (int m = 0; m < R; m++) {
            const c32 k4 = hG(g, f[0][m], pot_at(m, step), noise_at(m, step));
            st2(po, tile.b8(m), make_float2(fmaf(k4.x, 1.0f / 6.0f, f[1][m].x), fmaf(k4.y, 1.0f / 6.0f, f[1][m].y)));
        }
    } else if constexpr (MODE == PASS_AF) {
        // psibar = D^T abar + h J(psi_n)^T (D^T k1bar) (axis 0, after every other axis)
#pragma unroll
        for (int m = 0; m < R; m++) {
            const c32 pn = ld2(x0, tile.b8(m));
            const c32 g0b = f[1][m];
            const c32 r = hJT(g, pn, potential_at(m), g0b);
            if (vb) std_(vb, tile.b8(m), ldd(vb, tile.b8(m)) + (double)hImconj(g, g0b, pn));
            st2(ps, tile.b8(m), cadd(f[0][m], r));
        }
    } else {  // FIRST, D2, LF, XF, AS
#pragma unroll
        for (int m = 0; m < R; m++) {
            st2(pa, tile.b8(m), f[0][m]);
            st2(pb, tile.b8(m), f[1][m]);
        }
    }
}

// The fused passes of the adjoint step (default schedule: both fields at once).
// D2U, last axis: (A, B) -> D_last (A, B) = (a, k1) once the other axes are done; stored;
//   then u = a + k3 (the RK4 stages) and W' = D_last u, stored in psi.
// XAW, axis 0, once W' has been through every other axis: w = D_0 W' (the stage-4 input
//   D(a + k3)); then (A, B) = D_0^T (lam, h J(w)^T lam / 6), with V-bar += its term.
template <int N, int MODE, bool CONTIG, int LINES, bool NOISE, int RR>
__device__ __forceinline__ void axis_body_adjf(const GroupDev& g, int axis, const PassArgs& args, uint32_t bid,
                                               uint32_t nblk, c32* smem) {
    static_assert(adj_fused(MODE), "a fused adjoint pass");
    using F = FFTShape<N, RR>;
    constexpr int R = F::R, T = F::T;
    using L = LdsLayout<N, LINES, CONTIG, R>;
    using A = AxisLds<N, MODE, CONTIG, LINES, 0, RR, false>;
    c32* lds = smem;
    c32* tw = smem + A::BUF;
    c32* E = tw + N;
    stage_tables<F>(tw, E, g.tw[axis], g.E[axis]);
    const int t = CONTIG ? (int)(threadIdx.x % T) : (int)(threadIdx.x / LINES);
    const int l = CONTIG ? (int)(threadIdx.x / T) : (int)(threadIdx.x % LINES);
    const Tile<F, CONTIG, LINES> tile(g, axis, l, t, bid, nblk);
    const int64_t o = g.offset + tile.base;
    float2* __restrict__ ps = args.psi ? args.psi + o : nullptr;
    float2* __restrict__ pa = args.A ? args.A + o : nullptr;
    float2* __restrict__ pb = args.B ? args.B + o : nullptr;
    const float2* __restrict__ x0 = args.aux0 ? args.aux0 + o : nullptr;
    double* __restrict__ vb = args.vbar ? args.vbar + o : nullptr;
    const int64_t step = MODE == PASS_D2U ? read_step(args.step_off, args.step_base) : 0;
    const uint32_t iid = g.id_base + (uint32_t)tile.inst;
    const float* __restrict__ Vg = g.Vgrid ? g.Vgrid + tile.inst * g.M : nullptr;
    float V_other = 0.0f;
    {
        int x, y, z;
        unflatten(g, tile.j(0), x, y, z);
        const int c[3] = {x, y, z};
#pragma unroll
        for (int a = 0; a < 3; a++) {
            if (a == axis || a >= g.ndim) continue;
            const float xa = fmaf((float)c[a], g.dx[a], g.lo[a]);
            V_other = fmaf(g.half_trap[a] * xa, xa, V_other);
        }
    }
    const float ht_axis = g.half_trap[axis], lo_axis = g.lo[axis], dx_axis = g.dx[axis];
    auto potential_at = [&](int m) {
        const float xa = fmaf((float)(t + m * T), dx_axis, lo_axis);
        float Vp = fmaf(ht_axis * xa, xa, V_other);
        if (Vg) Vp += Vg[tile.j(m)];
        return Vp;
    };
    const c32 zero = make_float2(0.f, 0.f);
    c32 f[2][R];
    if constexpr (MODE == PASS_D2U) {
#pragma unroll
        for (int m = 0; m < R; m++) {
            f[0][m] = tile.active ? ld2(pa, tile.b8(m)) : zero;
            f[1][m] = tile.active ? ld2(pb, tile.b8(m)) : zero;
        }
        __syncthreads();  // tables staged
        propagate<F, L, 2>(f, t, l, lds, tw, E, false);
        c32(&u)[1][R] = *reinterpret_cast<c32(*)[1][R]>(&f[0]);
#pragma unroll
        for (int m = 0; m < R; m++) {
            if (tile.active) {
                st2(pa, tile.b8(m), f[0][m]);
                st2(pb, tile.b8(m), f[1][m]);
            }
            // u = a + k3 (the same arithmetic as the forward stages)
            c32 nz = zero;
            if constexpr (NOISE) {
                const float2 zz = noise_z(g, tile.j(m), iid, step);
                nz = make_float2(g.noise_c * zz.x, g.noise_c * zz.y);
            }
            const float Vp = potential_at(m);
            const c32 a = f[0][m], k1 = f[1][m];
            const c32 k2 = hG(g, make_float2(fmaf(0.5f, k1.x, a.x), fmaf(0.5f, k1.y, a.y)), Vp, nz);
            const c32 k3 = hG(g, make_float2(fmaf(0.5f, k2.x, a.x), fmaf(0.5f, k2.y, a.y)), Vp, nz);
            u[0][m] = cadd(a, k3);
        }
        propagate<F, L, 1>(u, t, l, lds, tw, E, false);
        if (!tile.active) return;  // after the last barrier
#pragma unroll
        for (int m = 0; m < R; m++) st2(ps, tile.b8(m), u[0][m]);
    } else {
        c32(&w)[1][R] = *reinterpret_cast<c32(*)[1][R]>(&f[1]);
#pragma unroll
        for (int m = 0; m < R; m++) w[0][m] = tile.active ? ld2(x0, tile.b8(m)) : zero;
        __syncthreads();  // tables staged
        propagate<F, L, 1>(w, t, l, lds, tw, E, false);
        // adjoint of psi' = D acc + k4/6, k4 = h G(w): (lam, wbar = h J(w)^T lam/6)
#pragma unroll
        for (int m = 0; m < R; m++) {
            const c32 lam = tile.active ? ld2(ps, tile.b8(m)) : zero;
            const c32 k4b = cscale(lam, 1.0f / 6.0f);
            const c32 wm = w[0][m];
            f[0][m] = lam;
            f[1][m] = hJT(g, wm, potential_at(m), k4b);
            if (vb && tile.active) std_(vb, tile.b8(m), ldd(vb, tile.b8(m)) + (double)hImconj(g, k4b, wm));
        }
        propagate<F, L, 2>(f, t, l, lds, tw, E, true);
        if (!tile.active) return;  // after the last barrier
#pragma unroll
        for (int m = 0; m < R; m++) {
            st2(pa, tile.b8(m), f[0][m]);
            st2(pb, tile.b8(m), f[1][m]);
        }
    }
}

// Passes with one thread per field (SEQ = 3): FIRST, D2, LF, XF, LAST2.
constexpr bool split_mode(int mode) {
    return mode == PASS_FIRST || mode == PASS_D2 || mode == PASS_LF || mode == PASS_XF || mode == PASS_LAST2;
}

// The pass on tile `bid` with one thread per field (SEQ = 3; 2 x T x LINES threads): the
// same arithmetic as axis_body with both fields at once, each field in its own half of
// the workgroup.
template <int N, int MODE, bool CONTIG, int LINES, bool NOISE, int RR, bool P64>
__device__ __forceinline__ void axis_body_split(const GroupDev& g, int axis, const PassArgs& args, uint32_t bid,
                                                uint32_t nblk,
                                                typename AxisLds<N, MODE, CONTIG, LINES, 3, RR, P64>::V* smem) {
    static_assert(split_mode(MODE), "a forward pass with two fields");
    using F = FFTShape<N, RR>;
    using V = typename std::conditional<P64, c64, c32>::type;
    constexpr int R = F::R, T = F::T;
    using L = LdsLayout<N, LINES, CONTIG, R>;
    using A = AxisLds<N, MODE, CONTIG, LINES, 3, RR, P64>;
    V* tw = smem + A::BUF;
    V* E = tw + N;
    if constexpr (P64)
        stage_tables<F>(tw, E, g.tw64[axis], g.E64[axis]);
    else
        stage_tables<F>(tw, E, g.tw[axis], g.E[axis]);
    const int tid = (int)(threadIdx.x % (unsigned)(T * LINES));
    const int q = (int)(threadIdx.x / (unsigned)(T * LINES));  // the field this thread carries
    V* lds = smem + q * L::SIZE;                                // its exchange buffer
    const V* partner = smem + (1 - q) * L::SIZE;                // the other field's
    const int t = CONTIG ? tid % T : tid / LINES;
    const int l = CONTIG ? tid / T : tid % LINES;
    const Tile<F, CONTIG, LINES> tile(g, axis, l, t, bid, nblk);
    const int64_t o = g.offset + tile.base;
    float2* __restrict__ ps = args.psi ? args.psi + o : nullptr;
    float2* __restrict__ pa = args.A ? args.A + o : nullptr;
    float2* __restrict__ pb = args.B ? args.B + o : nullptr;
    const int64_t step = read_step(args.step_off, args.step_base);
    const uint32_t iid = g.id_base + (uint32_t)tile.inst;
    const float* __restrict__ Vg = g.Vgrid ? g.Vgrid + tile.inst * g.M : nullptr;
    float V_other = 0.0f;
    {
        int x, y, z;
        unflatten(g, tile.j(0), x, y, z);
        const int c[3] = {x, y, z};
#pragma unroll
        for (int a = 0; a < 3; a++) {
            if (a == axis || a >= g.ndim) continue;
            const float xa = fmaf((float)c[a], g.dx[a], g.lo[a]);
            V_other = fmaf(g.half_trap[a] * xa, xa, V_other);
        }
    }
    const float ht_axis = g.half_trap[axis], lo_axis = g.lo[axis], dx_axis = g.dx[axis];
    auto pot_at = [&](int m, int64_t st) {
        const float xa = fmaf((float)(t + m * T), dx_axis, lo_axis);
        float Vp = fmaf(ht_axis * xa, xa, V_other);
        if (Vg) Vp += Vg[tile.j(m)];
        if constexpr (NOISE) {
            if (g.has_vnoise) Vp += vnoise(g, tile.j(m), iid, st);  // uniform
        }
        return Vp;
    };
    auto noise_at = [&](int m, int64_t st) {
        if constexpr (!NOISE) {
            return make_float2(0.f, 0.f);
        } else {
            const float2 zz = noise_z(g, tile.j(m), iid, st);
            return make_float2(g.noise_c * zz.x, g.noise_c * zz.y);
        }
    };
    const c32 zero = make_float2(0.f, 0.f);
    // the other half's field at this thread's elements, after this half's transform (the
    // buffers are free: the transforms' last exchanges are done)
    auto swap_in = [&](const c32 (&mine)[R], c32 (&theirs)[R]) {
#pragma unroll
        for (int m = 0; m < R; m++) lds[L::addr(l, t + m * T)] = widen(mine[m], V{});
        __syncthreads();
#pragma unroll
        for (int m = 0; m < R; m++) theirs[m] = narrow(partner[L::addr(l, t + m * T)]);
        __syncthreads();  // both halves have read before the next transform reuses the buffers
    };

    c32 f[1][R];
    if constexpr (MODE == PASS_FIRST) {
#pragma unroll
        for (int m = 0; m < R; m++) {
            const c32 psi = tile.active ? ld2(ps, tile.b8(m)) : zero;
            f[0][m] = q ? hG(g, psi, pot_at(m, step), noise_at(m, step)) : psi;
        }
    } else {
        const float2* src = q ? pb : pa;
#pragma unroll
        for (int m = 0; m < R; m++) f[0][m] = tile.active ? ld2(src, tile.b8(m)) : zero;
    }
    __syncthreads();  // tables staged
    propagate<F, L, 1>(f, t, l, lds, tw, E, false);

    if constexpr (MODE == PASS_LF || MODE == PASS_XF || MODE == PASS_LAST2) {
        c32 other[R];
        swap_in(f[0], other);
#pragma unroll
        for (int m = 0; m < R; m++) {
            const c32 f0 = q ? other[m] : f[0][m], f1 = q ? f[0][m] : other[m];
            if constexpr (MODE == PASS_LF) {
                // RK4 stages at the midpoint picture: (a, k1) -> (u, acc)
                const float Vp = pot_at(m, step);
                const c32 nz = noise_at(m, step);
                const c32 a = f0, k1 = f1;
                const c32 k2 = hG(g, make_float2(fmaf(0.5f, k1.x, a.x), fmaf(0.5f, k1.y, a.y)), Vp, nz);
                const c32 k3 = hG(g, make_float2(fmaf(0.5f, k2.x, a.x), fmaf(0.5f, k2.y, a.y)), Vp, nz);
                const float sx = k1.x * (1.0f / 6.0f) + (k2.x + k3.x) * (1.0f / 3.0f);
                const float sy = k1.y * (1.0f / 6.0f) + (k2.y + k3.y) * (1.0f / 3.0f);
                f[0][m] = q ? make_float2(a.x + sx, a.y + sy) : cadd(a, k3);
            } else if constexpr (MODE == PASS_XF) {
                // end of step n-1: psi_n = D acc + hG(D u)/6, then (psi_n, h G(psi_n))
                const c32 k4 = hG(g, f0, pot_at(m, step - 1), noise_at(m, step - 1));
                const c32 psi_n = make_float2(fmaf(k4.x, 1.0f / 6.0f, f1.x), fmaf(k4.y, 1.0f / 6.0f, f1.y));
                f[0][m] = q ? hG(g, psi_n, pot_at(m, step), noise_at(m, step)) : psi_n;
            } else {
                // LAST2: psi' = D acc + hG(D u)/6 (stored by the first half)
                const c32 k4 = hG(g, f0, pot_at(m, step), noise_at(m, step));
                f[0][m] = make_float2(fmaf(k4.x, 1.0f / 6.0f, f1.x), fmaf(k4.y, 1.0f / 6.0f, f1.y));
            }
        }
        if constexpr (MODE != PASS_LAST2) propagate<F, L, 1>(f, t, l, lds, tw, E, false);
    }

    if (!tile.active) return;  // after the last barrier
    if constexpr (MODE == PASS_LAST2) {
        if (q) return;
        float2* __restrict__ po = args.psi_out ? args.psi_out + o : ps;
#pragma unroll
        for (int m = 0; m < R; m++) st2(po, tile.b8(m), f[0][m]);
    } else {
        float2* dst = q ? pb : pa;
#pragma unroll
        for (int m = 0; m < R; m++) st2(dst, tile.b8(m), f[0][m]);
    }
}

// Threads of a workgroup of the pass.
template <int N, int LINES, int SEQ, int RR>
constexpr int pass_threads() { return FFTShape<N, RR>::T * LINES * (SEQ == 3 ? 2 : 1); }

// One group's pass: one workgroup per tile.
template <int N, int MODE, bool CONTIG, int LINES, bool NOISE, int SEQ, int RR, bool P64, int OCC>
__global__ void __launch_bounds__((pass_threads<N, LINES, SEQ, RR>())) __attribute__((amdgpu_waves_per_eu(OCC)))
k_axis(GroupDev g, int axis, PassArgs args) {
    using A = AxisLds<N, MODE, CONTIG, LINES, SEQ, RR, P64>;
    __shared__ typename A::V smem[A::ENTRIES];
    if constexpr (SEQ == 3) {
        if constexpr (split_mode(MODE))
            axis_body_split<N, MODE, CONTIG, LINES, NOISE, RR, P64>(g, axis, args, blockIdx.x, gridDim.x, smem);
    } else if constexpr (adj_fused(MODE)) {
        if constexpr (!P64 && SEQ == 0)
            axis_body_adjf<N, MODE, CONTIG, LINES, NOISE, RR>(g, axis, args, blockIdx.x, gridDim.x, smem);
    } else {
        axis_body<N, MODE, CONTIG, LINES, NOISE, SEQ, RR, P64>(g, axis, args, blockIdx.x, gridDim.x, smem);
    }
}

// LDS of a strided tile of w columns and nf fields must fit the 160 KiB of a CU.
constexpr bool fits_lds(int N, int w, int nf) { return (long)nf * N * w * 8 <= 128 * 1024; }

static inline int strided_lines(int N, int n0) {
    int w = N <= 256 ? 16 : (N == 512 ? 8 : 4);
    return w < n0 ? w : n0;
}

static inline int contig_lines(int N) {
    const int T = N < 16 ? 1 : N / 16;
    int l = 256 / T;
    return l < 1 ? 1 : l;
}



template <int N, int MODE, bool CONTIG, int LINES, int SEQ, int RR, bool P64, int OCC = 1>
static hipError_t go_axis(const GroupDev& g, int axis, const PassArgs& a, hipStream_t s) {
    int64_t blocks;
    if (CONTIG)
        blocks = (g.batch * (g.M >> g.log2n[0]) + LINES - 1) / LINES;
    else
        blocks = g.batch * (g.M >> g.log2n[axis]) / LINES;
    const dim3 grid((unsigned)blocks), block(pass_threads<N, LINES, SEQ, RR>());
    if constexpr (uses_rhs(MODE)) {
        if (g.has_noise) {
            hipLaunchKernelGGL((k_axis<N, MODE, CONTIG, LINES, true, SEQ, RR, P64, OCC>), grid, block, 0, s, g, axis, a);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((k_axis<N, MODE, CONTIG, LINES, false, SEQ, RR, P64, OCC>), grid, block, 0, s, g, axis, a);
    return hipGetLastError();
}

// passes that run only on axis 0 / only on the last (strided) axis
constexpr bool contig_only(int mode) {
    return mode == PASS_FIRST || mode == PASS_XF || mode == PASS_LAST2 || mode == PASS_XAW || mode == PASS_AF;
}
constexpr bool strided_only(int mode) {
    return mode == PASS_AS || mode == PASS_LF || mode == PASS_SI || mode == PASS_D2U;
}
// lengths with more than the default schedule compiled (the ones the workloads use)
constexpr bool tuned_length(int N) { return N >= 128 && N <= 512; }
// forward-step passes get the schedule variants; the adjoint passes use the default
constexpr bool tuned_mode(int mode) {
    return mode <= PASS_LAST2 || mode == PASS_LF || mode == PASS_XF || mode == PASS_SI;
}
// passes compiled with FP64 transforms (the forward step and the plain propagator)
constexpr bool f64_mode(int mode) { return tuned_mode(mode); }
// passes that read both fields of the pair from memory
constexpr bool loads_two_fields(int mode) {
    return mode == PASS_D2 || mode == PASS_LAST2 || mode == PASS_AS || mode == PASS_AF ||
           mode == PASS_LF || mode == PASS_XF;
}

constexpr int default_contig_lines(int N) { return N < 16 ? 256 : ((256 / (N / 16)) < 1 ? 1 : 256 / (N / 16)); }

// LDS bytes of a pass with FP64 transforms (8 values per thread): nf exchange buffers
// (LdsLayout) plus the two tables.
constexpr bool fits_lds64(int N, int lines, int nf, bool contig) {
    const long buf = contig ? (long)lines * (N + 1) : (long)lines * N;
    return ((long)nf * buf + 2L * N) * 16 <= 160L * 1024;
}

// Narrow tiles for small lattices (a single 512^2 lattice has only 512 lines per axis):
// one or two waves per workgroup, radix 8, both fields at once, so that a pass launches
// hundreds of workgroups instead of a hundred. Contiguous axis: a quarter or an eighth of
// the default lines; strided axes: one or two columns.
template <int N>
constexpr bool narrow_tile(bool contig, int lines) {
    const int T = N / 8;  // threads per line with 8 values per thread
    if (lines < 1 || T * lines < 64 || T * lines > 128) return false;
    if (contig) {
        const int dl = default_contig_lines(N);
        return lines == dl / 4 || lines == dl / 8;
    }
    return lines == 1 || lines == 2;
}

// Is schedule (lines, seq, rr) of pass MODE compiled for length N on the contiguous or a
// strided axis, with FP32 or FP64 transforms? Mirrors the instantiations in go_axis_n.
// rr = values per thread.
template <int N, int MODE>
constexpr bool schedule_compiled(bool contig, int lines, int seq, int rr, bool p64, int occ = 1) {
    constexpr int NF = fields_of(MODE);
    const bool tuned = tuned_length(N) && tuned_mode(MODE);
    if (seq < 0 || seq > 3) return false;
    if (seq == 3) {
        // one thread per field: radix 8 (LF and XF in FP32 also radix 16: with one field
        // per thread it fits four waves per SIMD), no occupancy hint, at most 1024 threads
        const bool r16 = rr == 16 && !p64 && (MODE == PASS_LF || MODE == PASS_XF);
        if (!split_mode(MODE) || !tuned || (rr != 8 && !r16) || occ != 1) return false;
        const int T = N / rr;
        if (T * lines * 2 > 1024) return false;
        if (p64 ? !fits_lds64(N, lines, 2, contig) : (!contig && !fits_lds(N, lines, 2))) return false;
        if (contig) {
            const int dl = default_contig_lines(N);
            return lines >= 1 && (lines == dl / 2 || lines == dl / 4 || (lines == dl / 8 && narrow_tile<N>(true, lines)));
        }
        return lines == 1 || lines == 2 || lines == 4 || lines == 8;
    }
    if (tuned && narrow_tile<N>(contig, lines)) return occ == 1 && seq == 0 && rr == 8;
    if (occ != 1) {
        // the four-wave variant: FP32, radix 8, both fields at once, tuned lengths
        if (occ != 4 || p64 || rr != 8 || seq != 0 || !tuned) return false;
        return schedule_compiled<N, MODE>(contig, lines, 0, 8, false, 1);
    }
    if (p64) {
        // radix 8 only (FP64 values take twice the registers), at most 512 threads
        if (!f64_mode(MODE) || rr != 8 || lines < 1) return false;
        if (seq && NF != 2) return false;
        if (seq == 2 && (!tuned || !loads_two_fields(MODE))) return false;
        const int nf = seq ? 1 : NF;
        const int T = N / (N < 8 ? N : 8);
        if (T * lines > 512 || !fits_lds64(N, lines, nf, contig)) return false;
        if (contig) {
            const int dl = default_contig_lines(N);
            if (tuned) return lines == dl || lines == dl / 2 || lines == dl / 4;
            return lines == (dl / 2 >= 1 ? dl / 2 : 1);
        }
        return lines == 4 || lines == 8 || lines == 16;
    }
    if (rr != 16 && !(rr == 8 && tuned)) return false;
    const int T = N / (N < rr ? N : rr);
    if (seq && (NF != 2 || !tuned)) return false;
    if (seq == 2 && !loads_two_fields(MODE)) return false;
    const int nf = seq ? 1 : NF;
    if (contig) {
        const int dl = default_contig_lines(N);  // 256 threads with 16 values per thread
        if (rr == 16 && lines == dl) return true;
        if (!tuned) return false;
        if (rr == 16) return lines == dl / 2 && lines >= 1;
        return (lines == dl || lines == dl / 2) && lines >= 1 && T * lines <= 1024;
    }
    if (lines != 4 && lines != 8 && lines != 16 && lines != 32) return false;
    if (T * lines > 1024 || !fits_lds(N, lines, nf)) return false;
    if (lines == 32 && !tuned) return false;
    return true;
}

template <int N, int MODE, bool CONTIG, int LINES, int RR, bool P64>
static hipError_t go_axis_sched_rr(const GroupDev& g, int axis, const PassArgs& a, hipStream_t s) {
    if constexpr (schedule_compiled<N, MODE>(CONTIG, LINES, 0, RR, P64, 4)) {
        if (a.occ == 4 && a.seq == 0) return go_axis<N, MODE, CONTIG, LINES, 0, RR, P64, 4>(g, axis, a, s);
    }
    if (a.occ != 0 && a.occ != 1) return hipErrorInvalidValue;
    if constexpr (schedule_compiled<N, MODE>(CONTIG, LINES, 3, RR, P64)) {
        if (a.seq == 3) return go_axis<N, MODE, CONTIG, LINES, 3, RR, P64>(g, axis, a, s);
    }
    if constexpr (schedule_compiled<N, MODE>(CONTIG, LINES, 2, RR, P64)) {
        if (a.seq == 2) return go_axis<N, MODE, CONTIG, LINES, 2, RR, P64>(g, axis, a, s);
    }
    if constexpr (schedule_compiled<N, MODE>(CONTIG, LINES, 1, RR, P64)) {
        if (a.seq == 1) return go_axis<N, MODE, CONTIG, LINES, 1, RR, P64>(g, axis, a, s);
    }
    if constexpr (schedule_compiled<N, MODE>(CONTIG, LINES, 0, RR, P64)) {
        if (a.seq == 0) return go_axis<N, MODE, CONTIG, LINES, 0, RR, P64>(g, axis, a, s);
    }
    return hipErrorInvalidValue;
}

template <int N, int MODE, bool CONTIG, int LINES, bool P64>
static hipError_t go_axis_sched(const GroupDev& g, int axis, const PassArgs& a, hipStream_t s) {
    if constexpr (P64) {
        if (a.radix == 8) return go_axis_sched_rr<N, MODE, CONTIG, LINES, 8, true>(g, axis, a, s);
        return hipErrorInvalidValue;
    } else {
        if (a.radix == 8) return go_axis_sched_rr<N, MODE, CONTIG, LINES, 8, false>(g, axis, a, s);
        if (a.radix == 0 || a.radix == 16) return go_axis_sched_rr<N, MODE, CONTIG, LINES, 16, false>(g, axis, a, s);
        return hipErrorInvalidValue;
    }
}

template <int N, int MODE, bool P64>
static hipError_t go_axis_np(const GroupDev& g, int axis, const PassArgs& a, hipStream_t s) {
    constexpr int CL = default_contig_lines(N);
    if (axis == 0) {
        if constexpr (strided_only(MODE)) {
            return hipErrorInvalidValue;
        } else {
            const int lines = a.lines ? a.lines : CL;
            if (lines == CL) return go_axis_sched<N, MODE, true, CL, P64>(g, axis, a, s);
            if constexpr (CL / 2 >= 1) {
                if (lines == CL / 2) return go_axis_sched<N, MODE, true, (CL / 2 >= 1 ? CL / 2 : 1), P64>(g, axis, a, s);
            }
            if constexpr (CL / 4 >= 1) {
                if (lines == CL / 4) return go_axis_sched<N, MODE, true, (CL / 4 >= 1 ? CL / 4 : 1), P64>(g, axis, a, s);
            }
            if constexpr (CL / 8 >= 1 && narrow_tile<N>(true, CL / 8)) {
                if (lines == CL / 8) return go_axis_sched<N, MODE, true, (CL / 8 >= 1 ? CL / 8 : 1), P64>(g, axis, a, s);
            }
            return hipErrorInvalidValue;
        }
    }
    if constexpr (contig_only(MODE)) {
        return hipErrorInvalidValue;
    } else {
        const int w = a.lines ? a.lines : strided_lines(N, g.n[0]);
        if (w > g.n[0]) return hipErrorInvalidValue;
        switch (w) {
            case 32: return go_axis_sched<N, MODE, false, 32, P64>(g, axis, a, s);
            case 16: return go_axis_sched<N, MODE, false, 16, P64>(g, axis, a, s);
            case 8: return go_axis_sched<N, MODE, false, 8, P64>(g, axis, a, s);
            case 4: return go_axis_sched<N, MODE, false, 4, P64>(g, axis, a, s);
            case 2: return go_axis_sched<N, MODE, false, 2, P64>(g, axis, a, s);
            case 1: return go_axis_sched<N, MODE, false, 1, P64>(g, axis, a, s);
            default: return hipErrorInvalidValue;
        }
    }
}

template <int N, int MODE>
static hipError_t go_axis_n(const GroupDev& g, int axis, const PassArgs& a, hipStream_t s) {
    if constexpr (f64_mode(MODE)) {
        if (a.f64) return go_axis_np<N, MODE, true>(g, axis, a, s);
    } else {
        if (a.f64) return hipErrorInvalidValue;
    }
    return go_axis_np<N, MODE, false>(g, axis, a, s);
}

template <int N>
static bool schedule_ok_n(int mode, bool contig, int lines, int seq, int rr, bool p64, int occ) {
    switch (mode) {
        case PASS_D1: return schedule_compiled<N, PASS_D1>(contig, lines, seq, rr, p64, occ);
        case PASS_D2: return schedule_compiled<N, PASS_D2>(contig, lines, seq, rr, p64, occ);
        case PASS_FIRST: return contig && schedule_compiled<N, PASS_FIRST>(contig, lines, seq, rr, p64, occ);
        case PASS_LAST2: return contig && schedule_compiled<N, PASS_LAST2>(contig, lines, seq, rr, p64, occ);
        case PASS_LF: return !contig && schedule_compiled<N, PASS_LF>(contig, lines, seq, rr, p64, occ);
        case PASS_XF: return contig && schedule_compiled<N, PASS_XF>(contig, lines, seq, rr, p64, occ);
        case PASS_SI: return !contig && schedule_compiled<N, PASS_SI>(contig, lines, seq, rr, p64, occ);
        default: return false;
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

}  // namespace rk4ip
