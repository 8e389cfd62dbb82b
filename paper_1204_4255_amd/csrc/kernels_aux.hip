// kernels_aux.hip -- FP64 reductions (norm, energy, overlap, ensemble moments), the
// graph step counter and the test kernels (Philox words, noise field, line FFTs).
#include "pass_common.h"

namespace rk4ip {

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
    using L = LdsLayout<N, LINES, true, F::R>;
    __shared__ c32 lds[L::SIZE];
    __shared__ c32 s_tw[N];
    stage_twiddles<F>(s_tw, tw);
    const int t = threadIdx.x % F::T;
    const int l = threadIdx.x / F::T;
    const int64_t line = (int64_t)blockIdx.x * LINES + l;
    const bool active = line < nlines;
    c32 v[1][F::R];
#pragma unroll
    for (int m = 0; m < F::R; m++) v[0][m] = active ? in[line * N + t + m * F::T] : make_float2(0.f, 0.f);
    __syncthreads();  // twiddles staged
    if (sign < 0)
        fft_line<F, -1, L, 1>(v, t, l, lds, s_tw);
    else
        fft_line<F, +1, L, 1>(v, t, l, lds, s_tw);
    if (active) {
#pragma unroll
        for (int m = 0; m < F::R; m++) out[line * N + t + m * F::T] = v[0][m];
    }
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
    using L = LdsLayout<N, LINES, CONTIG, F::R>;
    __shared__ c32 lds[L::SIZE];
    __shared__ c32 tw[N];
    __shared__ double red[FFTShape<N>::T * LINES][4];
    stage_tables<F, c32>(tw, nullptr, g.tw[axis], nullptr);
    const int t = CONTIG ? (int)(threadIdx.x % T) : (int)(threadIdx.x / LINES);
    const int l = CONTIG ? (int)(threadIdx.x / T) : (int)(threadIdx.x % LINES);
    const Tile<F, CONTIG, LINES> tile(g, axis, l, t, blockIdx.x, gridDim.x);
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
    __syncthreads();  // twiddles staged
    fft_line<F, -1, L, 1>(f, t, l, lds, tw);
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
            if constexpr (T * 16 <= 1024 && fits_lds(N, 16, 2))
                return go_diag<N, false, 16>(g, axis, psi, kscale, part, s);
            break;
        case 8:
            if constexpr (T * 8 <= 1024 && fits_lds(N, 8, 2)) return go_diag<N, false, 8>(g, axis, psi, kscale, part, s);
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
