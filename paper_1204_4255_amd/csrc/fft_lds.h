// fft_lds.h -- FFT of lines held in registers, exchanged through LDS (gfx950).
//
// The transforms between the spatial and spectral representations are FFTs applied
// along one lattice axis at a time (Dennis, Hope & Johnsson, arXiv:1204.4255, Sec. 3.2).
// Here a line of N = 2^p points is spread over T = N/R threads (R = min(N, 16) or
// min(N, 8) values per thread, kept in VGPRs). The transform is a Stockham autosort
// sequence of radix-R stages followed by at most one smaller stage; butterflies run in
// registers and the data move between stages through LDS. Thread t holds elements
// t + m*T (m = 0..R-1) both before the forward and after the inverse transform, which
// is exactly the pattern of a coalesced global load of the line, so no LDS round trip
// is needed at the ends.
//
// Forward transforms use e^{-2 pi i j m / N}, the inverse e^{+...}; neither is
// normalised. Twiddles e^{-2 pi i t / N} come from a table computed in FP64, staged in
// LDS by the caller in the stage-major order of FFTShape::tw_off (stage_twiddles). Every function is generic over the complex type: float2 for the
// complex64 transforms, double2 for the FP64-transform precision form (same code, the
// table and the LDS buffer in the same type).
#pragma once
#include <hip/hip_runtime.h>

namespace rk4ip {

typedef float2 c32;
typedef double2 c64;

__device__ __forceinline__ c32 cadd(c32 a, c32 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ c32 csub(c32 a, c32 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ c32 cscale(c32 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ c32 cmul(c32 a, c32 b) {
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ c32 cconj(c32 a) { return make_float2(a.x, -a.y); }

// The same operations in FP64 (the transforms of the FP64-transform precision form).
__device__ __forceinline__ c64 cadd(c64 a, c64 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ c64 csub(c64 a, c64 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ c64 cmul(c64 a, c64 b) {
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ c64 cconj(c64 a) { return make_double2(a.x, -a.y); }

__device__ __forceinline__ c32 mk(float x, float y, c32) { return make_float2(x, y); }
__device__ __forceinline__ c64 mk(double x, double y, c64) { return make_double2(x, y); }

// multiply by i^{s}: s = -1 -> -i z, s = +1 -> i z
template <int S, class V>
__device__ __forceinline__ V mul_i(V z) {
    return S < 0 ? mk(z.y, -z.x, z) : mk(-z.y, z.x, z);
}

// cos and sin of pi/8 and cos(pi/4) in the working precision: the FP32 constants are the
// correctly rounded values, the FP64 ones carry 17 significant digits.
template <class Sc>
struct W16;
template <>
struct W16<float> {
    static constexpr float C1 = 0.92387953251128674f;  // cos(pi/8)
    static constexpr float S1 = 0.38268343236508977f;  // sin(pi/8)
    static constexpr float H = 0.70710678118654752f;   // cos(pi/4)
};
template <>
struct W16<double> {
    static constexpr double C1 = 0.92387953251128674;
    static constexpr double S1 = 0.38268343236508977;
    static constexpr double H = 0.70710678118654752;
};

template <int S, int K, class V>
__device__ __forceinline__ V w16_mul(V z) {
    // z * e^{S 2 pi i K / 16}
    using Sc = decltype(z.x);
    using C = W16<Sc>;
    constexpr int k = ((K % 16) + 16) % 16;
    if constexpr (k == 0) {
        return z;
    } else if constexpr (k == 4) {
        return mul_i<S>(z);
    } else if constexpr (k == 8) {
        return mk(-z.x, -z.y, z);
    } else if constexpr (k == 12) {
        return mul_i<-S>(z);
    } else if constexpr (k == 2 || k == 6 || k == 10 || k == 14) {
        // (1 + S i)/sqrt2 rotated by multiples of i
        constexpr Sc c = (k == 2 || k == 14) ? C::H : -C::H;
        constexpr Sc s = (k == 2 || k == 6) ? C::H : -C::H;  // sin(2 pi k/16) sign
        const Sc ss = S * s;
        return mk(fma(z.x, c, -z.y * ss), fma(z.x, ss, z.y * c), z);
    } else {
        // odd k: cos/sin of k pi / 8
        constexpr Sc cs[16] = {1, C::C1, C::H, C::S1, 0, -C::S1, -C::H, -C::C1,
                               -1, -C::C1, -C::H, -C::S1, 0, C::S1, C::H, C::C1};
        constexpr Sc sn[16] = {0, C::S1, C::H, C::C1, 1, C::C1, C::H, C::S1,
                               0, -C::S1, -C::H, -C::C1, -1, -C::C1, -C::H, -C::S1};
        const Sc c = cs[k];
        const Sc s = S * sn[k];
        return mk(fma(z.x, c, -z.y * s), fma(z.x, s, z.y * c), z);
    }
}

// In-register DFTs with natural-order input and output: y_k = sum_j x_j e^{S 2 pi i jk/r}.
template <int S, class V>
__device__ __forceinline__ void dft2(V& a, V& b) {
    V t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

template <int S, class V>
__device__ __forceinline__ void dft4(V& x0, V& x1, V& x2, V& x3) {
    V s02 = cadd(x0, x2), d02 = csub(x0, x2);
    V s13 = cadd(x1, x3), d13 = mul_i<S>(csub(x1, x3));
    x0 = cadd(s02, s13);
    x2 = csub(s02, s13);
    x1 = cadd(d02, d13);
    x3 = csub(d02, d13);
}

template <int R, int S>
struct DFT;

template <int S>
struct DFT<2, S> {
    template <class V>
    __device__ __forceinline__ static void run(V (&x)[2]) { dft2<S>(x[0], x[1]); }
};

template <int S>
struct DFT<4, S> {
    template <class V>
    __device__ __forceinline__ static void run(V (&x)[4]) { dft4<S>(x[0], x[1], x[2], x[3]); }
};

// 8 = 2 x 4: j = j1 + 2 j2, k = 4 k1 + k2
template <int S>
struct DFT<8, S> {
    template <class V>
    __device__ __forceinline__ static void run(V (&x)[8]) {
        dft4<S>(x[0], x[2], x[4], x[6]);  // j1 = 0 -> Y[0][k2] in x[0,2,4,6]
        dft4<S>(x[1], x[3], x[5], x[7]);  // j1 = 1 -> Y[1][k2] in x[1,3,5,7]
        x[3] = w16_mul<S, 2>(x[3]);       // W8^{k2}, k2 = 1..3
        x[5] = w16_mul<S, 4>(x[5]);
        x[7] = w16_mul<S, 6>(x[7]);
        dft2<S>(x[0], x[1]);  // k2 = 0 -> X[0], X[4]
        dft2<S>(x[2], x[3]);  // k2 = 1 -> X[1], X[5]
        dft2<S>(x[4], x[5]);  // k2 = 2 -> X[2], X[6]
        dft2<S>(x[6], x[7]);  // k2 = 3 -> X[3], X[7]
        V y[8] = {x[0], x[2], x[4], x[6], x[1], x[3], x[5], x[7]};
#pragma unroll
        for (int i = 0; i < 8; i++) x[i] = y[i];
    }
};

// 16 = 4 x 4: j = j1 + 4 j2, k = 4 k1 + k2; W16^{jk} = W4^{j1 k1} W16^{j1 k2} W4^{j2 k2}
template <int S>
struct DFT<16, S> {
    template <class V>
    __device__ __forceinline__ static void run(V (&x)[16]) {
        // step A: for each j1, DFT4 over j2 of x[j1 + 4 j2] -> Y[j1][k2] stored at x[j1 + 4 k2]
        dft4<S>(x[0], x[4], x[8], x[12]);
        dft4<S>(x[1], x[5], x[9], x[13]);
        dft4<S>(x[2], x[6], x[10], x[14]);
        dft4<S>(x[3], x[7], x[11], x[15]);
        // step B: Y[j1][k2] *= W16^{j1 k2}
        x[5] = w16_mul<S, 1>(x[5]);
        x[9] = w16_mul<S, 2>(x[9]);
        x[13] = w16_mul<S, 3>(x[13]);
        x[6] = w16_mul<S, 2>(x[6]);
        x[10] = w16_mul<S, 4>(x[10]);
        x[14] = w16_mul<S, 6>(x[14]);
        x[7] = w16_mul<S, 3>(x[7]);
        x[11] = w16_mul<S, 6>(x[11]);
        x[15] = w16_mul<S, 9>(x[15]);
        // step C: for each k2, DFT4 over j1 of Y[j1][k2] = x[j1 + 4 k2] -> X[4 k1 + k2]
        dft4<S>(x[0], x[1], x[2], x[3]);
        dft4<S>(x[4], x[5], x[6], x[7]);
        dft4<S>(x[8], x[9], x[10], x[11]);
        dft4<S>(x[12], x[13], x[14], x[15]);
        // now x[k1 + 4 k2] holds X[4 k1 + k2]: transpose the 4 x 4 index
        V y[16];
#pragma unroll
        for (int k1 = 0; k1 < 4; k1++)
#pragma unroll
            for (int k2 = 0; k2 < 4; k2++) y[4 * k1 + k2] = x[k1 + 4 * k2];
#pragma unroll
        for (int i = 0; i < 16; i++) x[i] = y[i];
    }
};

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

// Shape of the transform of a line of N points with at most RR values per thread: a
// sequence of radix-R stages (R = min(N, RR)) and at most one smaller last stage.
template <int N, int RR = 16>
struct FFTShape {
    static_assert(N >= 8 && (N & (N - 1)) == 0, "N must be a power of two >= 8");
    static_assert(RR == 8 || RR == 16, "8 or 16 values per thread");
    static constexpr int NN = N;
    static constexpr int R = N < RR ? N : RR;   // values per thread
    static constexpr int T = N / R;             // threads per line
    static constexpr int LR = ilog2(R);
    static constexpr int S = N < RR ? 0 : ilog2(N) / LR;        // full radix-R stages
    static constexpr int Q = N < RR ? N : (N >> (LR * S));      // last radix (1 = none)
    static constexpr int NSTAGES = S + (Q > 1 ? 1 : 0);
    // radix and Ns (product of earlier radices) of stage i
    __host__ __device__ static constexpr int radix(int i) { return (N < RR) ? N : (i < S ? R : Q); }
    __host__ __device__ static constexpr int ns(int i) { return i == 0 ? 1 : ns(i - 1) * radix(i - 1); }
    // first entry of stage i's twiddles in the stage-major table (stage 0 needs none): the
    // factor e^{-2 pi i bm k step / N} of butterfly bm and input k >= 1 of stage i sits at
    // tw_off(i) + (k - 1) ns(i) + bm, so the butterflies of a wavefront read consecutive
    // entries. The table has N - 1 entries.
    __host__ __device__ static constexpr int tw_off(int i) {
        return i <= 1 ? 0 : tw_off(i - 1) + ns(i - 1) * (radix(i - 1) - 1);
    }
};

// LDS layout of an exchange buffer that holds `LINES` lines of N complex values, for a
// transform with R values per thread.
//  * ROWMAJOR (lines contiguous; the threads of a line are adjacent lanes): with R = 8,
//    a one-slot row pad and the element index XORed with its own bits 3-6 in bits 0-3,
//    which removes most bank conflicts of the radix-8 exchanges (checked on the host
//    against 32 banks x 16 lanes and 64 banks x 32 lanes per cycle for 8-byte accesses);
//    otherwise one pad slot every 16 values.
//  * element-major with the line index fastest (adjacent lanes hold adjacent lines, the
//    columns of a strided axis). Padding that removes the remaining 2-way conflicts of the
//    first exchange costs more address arithmetic than it saves in these VALU-bound
//    passes, so there is none.
template <int N, int LINES, bool ROWMAJOR, int R = 16>
struct LdsLayout {
    static constexpr bool ROWS = ROWMAJOR;
    static constexpr bool SWZ = ROWMAJOR && R == 8 && N >= 16;
    static constexpr int ROW = SWZ ? N + 1 : N + (N >= 16 ? N / 16 : 0);
    static constexpr int SIZE = ROWMAJOR ? LINES * ROW : LINES * N;
    __device__ __forceinline__ static int addr(int line, int e) {
        if constexpr (ROWMAJOR) {
            if constexpr (SWZ) {
                return line * ROW + (e ^ ((e >> 3) & 15 & (N - 1)));
            } else {
                return line * ROW + e + (N >= 16 ? (e >> 4) : 0);
            }
        } else {
            return e * LINES + line;
        }
    }
};

// Twiddles of every stage of F in the stage-major order of FFTShape::tw_off, built from
// the canonical table tw[j] = e^{-2 pi i j / N}. All threads of the block call it; the
// caller synchronises before the first transform.
template <class F, int STAGE, class V>
__device__ __forceinline__ void stage_twiddles_from(V* s_tw, const V* __restrict__ tw) {
    if constexpr (STAGE < F::NSTAGES) {
        constexpr int ns = F::ns(STAGE), r = F::radix(STAGE), step = F::NN / (ns * r);
        for (int i = threadIdx.x; i < ns * (r - 1); i += blockDim.x) {
            const int k = i / ns + 1, bm = i - (k - 1) * ns;
            s_tw[F::tw_off(STAGE) + i] = tw[bm * k * step];
        }
        stage_twiddles_from<F, STAGE + 1>(s_tw, tw);
    }
}

template <class F, class V>
__device__ __forceinline__ void stage_twiddles(V* s_tw, const V* __restrict__ tw) {
    stage_twiddles_from<F, 1>(s_tw, tw);
}

// One Stockham stage on the registers of one thread: U = R/radix butterflies,
// butterfly u is b = t + T u with inputs v[u*radix + k] = x[b + k N/radix].
template <class F, int S, int STAGE, class V>
__device__ __forceinline__ void fft_stage(V (&v)[F::R], int t, const V* __restrict__ tw) {
    constexpr int r = F::radix(STAGE);
    constexpr int ns = F::ns(STAGE);
    constexpr int U = F::R / r;
#pragma unroll
    for (int u = 0; u < U; u++) {
        V x[r];
#pragma unroll
        for (int k = 0; k < r; k++) x[k] = v[u * r + k];
        if constexpr (ns > 1) {
            const int b = t + F::T * u;
            const int bm = b & (ns - 1);
#pragma unroll
            for (int k = 1; k < r; k++) {
                V w = tw[F::tw_off(STAGE) + (k - 1) * ns + bm];
                if constexpr (S > 0) w = cconj(w);
                x[k] = cmul(x[k], w);
            }
        }
        DFT<r, S>::run(x);
#pragma unroll
        for (int k = 0; k < r; k++) v[u * r + k] = x[k];
    }
}

// Order this wave's LDS accesses on either side: the wave's LDS instructions execute in
// order, so what its lanes wrote before is what its lanes read after, with no workgroup
// barrier (the fences keep the compiler from moving LDS accesses across).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The exchange of a line whose threads are consecutive lanes of one wave (row-major
// buffer, at most 64 threads per line; every kernel with a row-major buffer gives thread
// t of line l the index l T + t) touches LDS that only that wave uses: a wave-level sync
// suffices. Otherwise the line spans waves and needs the workgroup barrier.
template <class F, class L>
__device__ __forceinline__ void exchange_sync() {
    if constexpr (L::ROWS && F::T <= 64) {
        wave_lds_sync();
    } else {
        __syncthreads();
    }
}

// Write the outputs of stage STAGE to LDS and read the inputs of stage STAGE+1.
template <class F, int STAGE, class L, int NF, class V>
__device__ __forceinline__ void fft_exchange(V (&v)[NF][F::R], int t, int line, V* lds) {
    constexpr int N = F::NN;
    constexpr int r = F::radix(STAGE);
    constexpr int ns = F::ns(STAGE);
    constexpr int U = F::R / r;
    constexpr int r2 = F::radix(STAGE + 1);
    constexpr int U2 = F::R / r2;
#pragma unroll
    for (int f = 0; f < NF; f++) {
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int b = t + F::T * u;
            const int base = (b / ns) * ns * r + (b & (ns - 1));
#pragma unroll
            for (int k = 0; k < r; k++) lds[f * L::SIZE + L::addr(line, base + k * ns)] = v[f][u * r + k];
        }
    }
    exchange_sync<F, L>();
#pragma unroll
    for (int f = 0; f < NF; f++) {
#pragma unroll
        for (int u = 0; u < U2; u++) {
            const int b = t + F::T * u;
#pragma unroll
            for (int k = 0; k < r2; k++) v[f][u * r2 + k] = lds[f * L::SIZE + L::addr(line, b + k * (N / r2))];
        }
    }
    exchange_sync<F, L>();
}

// After the last stage, register u*Q + k holds element t + T (u + k R/Q); put element
// t + T m into register m.
template <class F, class V>
__device__ __forceinline__ void fft_natural_order(V (&v)[F::R]) {
    constexpr int r = F::radix(F::NSTAGES - 1);
    constexpr int U = F::R / r;
    if constexpr (U > 1) {
        V y[F::R];
#pragma unroll
        for (int u = 0; u < U; u++)
#pragma unroll
            for (int k = 0; k < r; k++) y[u + k * U] = v[u * r + k];
#pragma unroll
        for (int i = 0; i < F::R; i++) v[i] = y[i];
    }
}

// Stage i of a transform of NF fields at once: the register half of stage i, then the
// exchange into stage i+1.
template <class F, int S, int STAGE, class L, int NF, class V>
__device__ __forceinline__ void fft_stages_from(V (&v)[NF][F::R], int t, int line, V* lds,
                                                const V* __restrict__ tw) {
#pragma unroll
    for (int f = 0; f < NF; f++) fft_stage<F, S, STAGE>(v[f], t, tw);
    if constexpr (STAGE + 1 < F::NSTAGES) {
        fft_exchange<F, STAGE, L, NF>(v, t, line, lds);
        fft_stages_from<F, S, STAGE + 1, L, NF>(v, t, line, lds, tw);
    }
}

// Full transform of NF lines (one per field) owned by this thread group. On entry and
// on exit thread t holds element t + T m in v[f][m]. S = -1 forward, +1 inverse. F is the
// FFTShape (length and values per thread). All threads of the block must call this
// together (it contains barriers, workgroup-wide unless the line sits in one wave).
template <class F, int S, class L, int NF, class V>
__device__ __forceinline__ void fft_line(V (&v)[NF][F::R], int t, int line, V* lds,
                                         const V* __restrict__ tw) {
    fft_stages_from<F, S, 0, L, NF>(v, t, line, lds, tw);
#pragma unroll
    for (int f = 0; f < NF; f++) fft_natural_order<F>(v[f]);
}

}  // namespace rk4ip
