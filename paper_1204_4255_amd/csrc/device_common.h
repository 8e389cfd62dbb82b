// device_common.h -- per-group parameters, counter-based noise and the pointwise
// right-hand side used by every RK4IP kernel.
//
// Right-hand side (Dennis, Hope & Johnsson, arXiv:1204.4255, Sec. 3.6 eq. (7) and
// Sec. 4.1 eq. (9)): G(psi) = -i (V + g |psi|^2) psi + sigma xi, evaluated in FP32.
// Noise (Sec. 3.5, Wiener noise, Stratonovich form): xi is drawn from Philox4x32-10
// (Salmon, Moraes, Dror, Shaw, SC'11) and is a pure function of (seed, instance, step,
// point), regenerated wherever it is needed instead of being stored.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_lds.h"

namespace rk4ip {

// Everything a kernel needs to know about one group of same-shape instances.
struct GroupDev {
    int ndim;
    int n[3];
    int log2n[3];
    int64_t M;          // points per instance
    int64_t batch;
    int64_t offset;     // index of the group's first point in the concatenated field
    float lo[3];
    float dx[3];
    float half_trap[3]; // V = sum half_trap[a] x_a^2 (+ Vgrid)
    float h;            // time step
    float gnl;
    float noise_c;      // h sigma / sqrt(2 h dV): multiplies a complex normal with E|z|^2 = 2
    float xi_scale;     // 1 / sqrt(2 h dV): xi = xi_scale z
    float inv_n[3];     // 1/n_a (exact)
    uint32_t seed_lo, seed_hi, id_base;
    int has_noise;
    const float* Vgrid;      // [batch][M] or nullptr
    const float2* E[3];      // per axis: (E_a - 1)/n_a, see mul_dE
    const float2* tw[3];     // per axis: e^{-2 pi i t / n_a}
    const double2* E64[3];   // the same tables in FP64 (FP64-transform plans, else null)
    const double2* tw64[3];
    int noise_sub;           // noise of a step = normalised sum of this many finer draws
    float inv_sqrt_sub;      // 1/sqrt(noise_sub)
    int has_vnoise;          // real Wiener noise in the potential (1D groups)
    float vnoise_c;          // sigma_V / sqrt(h dV): multiplies a unit real normal
    const float2* convK;     // [n] (FFT of the non-local kernel) dV / n (1D groups), or null
    const float2* E2;        // [n] (e^{L h} - 1)/n of axis 0 (1D Fourier groups: the k-space line
                             // step), else null
    const double2* pairT1;   // [n] cosine / sine line through its reordered transform: (A - 1)/n and
    const double2* pairT2;   // B/n of the mode-pairing propagator, FP64 (else null)
    float2* K;               // [batch][n] the k-space state of a 1D group run by the k-space line
                             // step (kept between the launches of a run), else null
    int basis;               // 1D: 0 Fourier; 1 cosine, 2 sine (n[0] is then the length of the
                             // even / odd extension, twice the stored points)
};

// ---------------------------------------------------------------- Philox4x32-10
struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; r++) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c.x;
        const uint32_t hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z);
        U4 n;
        n.x = hi1 ^ c.y ^ k0;
        n.y = lo1;
        n.z = hi0 ^ c.w ^ k1;
        n.w = lo0;
        c = n;
    }
    return c;
}

// Counter of the pair of points (2q, 2q+1) of an instance at a step, tag 0 (dynamics).
// Counter of point j of instance `inst` at `step`; the tag (top byte of the last word)
// separates streams: 0 the additive noise, 3 the noise in the potential.
__device__ __forceinline__ U4 noise_counter(int64_t j, uint32_t inst, int64_t step, uint32_t tag = 0) {
    U4 c;
    const uint64_t q = (uint64_t)j >> 1;
    const uint64_t st = (uint64_t)step;
    c.x = (uint32_t)q;
    c.y = inst;
    c.z = (uint32_t)st;
    c.w = (tag << 24) | (uint32_t)((st >> 32) & 0xFFFFFFu);
    return c;
}

// Box-Muller on two 24-bit uniforms: u1 in (0,1], u2 in [0,1). The complex normal
// z = rad (cos, sin)(2 pi u2), E|z|^2 = 2, as its radius and unit phasor.
__device__ __forceinline__ void box_muller(uint32_t ra, uint32_t rb, float& rad, float& c, float& s) {
    const float u1 = (float)((ra >> 8) + 1u) * 5.9604644775390625e-08f;  // 2^-24, exact
    const float u2 = (float)(rb >> 8) * 5.9604644775390625e-08f;
    rad = sqrtf(-2.0f * logf(u1));
    sincospif(2.0f * u2, &s, &c);
}

// Unit complex normal (E|z|^2 = 2) for point j of instance `inst` at `step`. With S noise
// substeps it is the sum of the normals of steps step*S ... step*S + S - 1 of a run with
// step h/S, divided by sqrt(S): one Wiener path sampled at several step sizes. The sum is
// written as explicit FMAs so that every kernel rounds it the same way (S = 1: the
// rounded product rad * cos, as a single draw).
__device__ __forceinline__ float2 noise_z(const GroupDev& g, int64_t j, uint32_t inst, int64_t step) {
    const int S = g.noise_sub;
    if (S == 1) {
        // one draw per step (the common case; the same value as the loop below)
        const U4 r = philox4x32_10(noise_counter(j, inst, step), g.seed_lo, g.seed_hi);
        float rad, c, sn;
        if (j & 1)
            box_muller(r.z, r.w, rad, c, sn);
        else
            box_muller(r.x, r.y, rad, c, sn);
        return make_float2(rad * c, rad * sn);
    }
    float2 acc = make_float2(0.f, 0.f);
    for (int s = 0; s < S; s++) {
        const U4 r = philox4x32_10(noise_counter(j, inst, step * S + s), g.seed_lo, g.seed_hi);
        float rad, c, sn;
        if (j & 1)
            box_muller(r.z, r.w, rad, c, sn);
        else
            box_muller(r.x, r.y, rad, c, sn);
        acc.x = fmaf(rad, c, acc.x);
        acc.y = fmaf(rad, sn, acc.y);
    }
    return make_float2(acc.x * g.inv_sqrt_sub, acc.y * g.inv_sqrt_sub);
}

// The unit complex normals of R points j(m) = j0 + m S (S even, m < R) of one lane, when
// the partner lane (lane ^ 1) holds the points j(m) ^ 1: a Philox block feeds the pair of
// points (2q, 2q + 1), so the even lane draws the blocks of m < R/2 and the odd lane those
// of m >= R/2, and each hands the partner the two words it needs. The same integers and the
// same arithmetic as noise_z with one draw per step (bitwise the same values), half the
// Philox work. All lanes of the wavefront must call it together.
template <int R>
__device__ __forceinline__ void noise_z_pairs(const GroupDev& g, int64_t j0, int64_t S, uint32_t inst, int64_t step,
                                              float2 (&z)[R]) {
    static_assert(R % 2 == 0, "pairs of elements");
    const bool odd = (j0 & 1) != 0;
    const int64_t jb = j0 + (odd ? (int64_t)(R / 2) * S : 0);  // first element this lane draws for
    uint32_t lo_w[R / 2][2], hi_w[R / 2][2];  // words of element k and of element k + R/2
#pragma unroll
    for (int k = 0; k < R / 2; k++) {
        const U4 r = philox4x32_10(noise_counter(jb + k * S, inst, step), g.seed_lo, g.seed_hi);
        // keep the words of this lane's own point, send the partner's
        const uint32_t keep0 = odd ? r.z : r.x, keep1 = odd ? r.w : r.y;
        const uint32_t send0 = odd ? r.x : r.z, send1 = odd ? r.y : r.w;
        const uint32_t got0 = (uint32_t)__shfl_xor((int)send0, 1);
        const uint32_t got1 = (uint32_t)__shfl_xor((int)send1, 1);
        lo_w[k][0] = odd ? got0 : keep0;
        lo_w[k][1] = odd ? got1 : keep1;
        hi_w[k][0] = odd ? keep0 : got0;
        hi_w[k][1] = odd ? keep1 : got1;
    }
#pragma unroll
    for (int m = 0; m < R; m++) {
        const uint32_t a = m < R / 2 ? lo_w[m % (R / 2)][0] : hi_w[m % (R / 2)][0];
        const uint32_t b = m < R / 2 ? lo_w[m % (R / 2)][1] : hi_w[m % (R / 2)][1];
        float rad, c, sn;
        box_muller(a, b, rad, c, sn);
        z[m] = make_float2(rad * c, rad * sn);
    }
}

// The noise of the potential at point j (in units of the potential): sigma_V eta with
// eta = Re(z)/sqrt(h dV), z the complex normal of counter tag 3, summed over the noise
// substeps like noise_z (explicit FMAs for the same reason).
__device__ __forceinline__ float vnoise(const GroupDev& g, int64_t j, uint32_t inst, int64_t step) {
    const int S = g.noise_sub;
    float acc = 0.f;
    for (int s = 0; s < S; s++) {
        const U4 r = philox4x32_10(noise_counter(j, inst, step * S + s, 3u), g.seed_lo, g.seed_hi);
        float rad, c, sn;
        if (j & 1)
            box_muller(r.z, r.w, rad, c, sn);
        else
            box_muller(r.x, r.y, rad, c, sn);
        acc = fmaf(rad, c, acc);
    }
    return acc * g.inv_sqrt_sub * g.vnoise_c;
}

// Trap potential at lattice indices (x, y, z).
__device__ __forceinline__ float trap_V(const GroupDev& g, int ix, int iy, int iz) {
    float v = 0.0f;
    const float x = fmaf((float)ix, g.dx[0], g.lo[0]);
    v = fmaf(g.half_trap[0] * x, x, v);
    if (g.ndim > 1) {
        const float y = fmaf((float)iy, g.dx[1], g.lo[1]);
        v = fmaf(g.half_trap[1] * y, y, v);
    }
    if (g.ndim > 2) {
        const float z = fmaf((float)iz, g.dx[2], g.lo[2]);
        v = fmaf(g.half_trap[2] * z, z, v);
    }
    return v;
}

// h G(phi) = -i h (V + g |phi|^2) phi + hnz, with hnz = noise_c * z (already scaled). The last products
// and the noise add are one explicit FMA, so every kernel that evaluates G (the fused
// passes and the ones that open and close a run) rounds it identically and split runs
// stay bitwise equal to whole ones.
__device__ __forceinline__ c32 hG(const GroupDev& g, c32 phi, float V, c32 hnz) {
    const float m2 = fmaf(phi.x, phi.x, phi.y * phi.y);
    const float w = g.h * fmaf(g.gnl, m2, V);
    return make_float2(fmaf(w, phi.y, hnz.x), fmaf(-w, phi.x, hnz.y));
}

// Transposes for the discrete adjoint (not in the paper). G is R-linear in (phi, conj phi):
// dG = A dphi + B conj(dphi) - i dV phi with A = -i (V + 2 g |phi|^2), B = -i g phi^2. With the
// real inner product <x, y> = Re sum conj(x) y its transpose is conj(A) lam + B conj(lam),
// and the potential gradient picks up Im(conj(lam) phi).
__device__ __forceinline__ c32 hJT(const GroupDev& g, c32 phi, float V, c32 lam) {
    const float m2 = fmaf(phi.x, phi.x, phi.y * phi.y);
    const float ar = fmaf(2.0f * g.gnl, m2, V);
    const float P = fmaf(phi.x, phi.x, -phi.y * phi.y);
    const float Q = 2.0f * phi.x * phi.y;
    const float cx = fmaf(P, lam.x, Q * lam.y);
    const float cy = fmaf(Q, lam.x, -P * lam.y);
    return make_float2(g.h * fmaf(g.gnl, cy, -ar * lam.y), g.h * fmaf(ar, lam.x, -g.gnl * cx));
}

// h Im(conj(lam) phi)
__device__ __forceinline__ float hImconj(const GroupDev& g, c32 lam, c32 phi) {
    return g.h * fmaf(lam.x, phi.y, -lam.y * phi.x);
}

// Spectral multiplier of the propagator in delta form. The table holds
// (E_a - 1)/n_a = ((e cos(theta) - 1)/n, -e sin(theta)/n) with e the damping factor (axis 0
// only) and theta = alpha k^2 h/2, computed in FP64 and rounded once. D_a is applied as
//     f + F_a^{-1}[ (E_a - 1)/n F_a f ],
// so the rounding error of the transform pair is scaled by |E_a - 1|, which is small on
// the modes that carry the field, and the rounded multiplier has no modulus bias.
__device__ __forceinline__ c32 mul_dE(c32 F, float2 cs) { return cmul(F, cs); }
__device__ __forceinline__ c32 mul_dE_adj(c32 F, float2 cs) { return cmul(F, make_float2(cs.x, -cs.y)); }

}  // namespace rk4ip
