// launch.h -- host-side entry points of the kernels in kernels.hip (library internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rk4ip {

struct GroupDev;

// Kinds of axis pass (see pass_common.h for the data flow of each). FIRST, D2, LF, XF and
// LAST2 make the forward step; D2U, XAW, AS and AF are the extra passes of the adjoint step.
enum PassMode {
    PASS_D1 = 0,
    PASS_D2 = 1,
    PASS_FIRST = 2,
    PASS_LAST2 = 4,
    PASS_AS = 7,
    PASS_AF = 8,
    PASS_LF = 9,   // last axis: D, the RK4 stage epilogue, D again
    PASS_XF = 10,  // axis 0: D, the end of one step, the start of the next, D again
    PASS_SI = 11,  // last axis, semi-implicit step: D, the midpoint iteration, D again
    PASS_D2U = 12, // adjoint recompute, last axis: (A, B) -> D (a, k1), then u = a + k3 -> D u
    PASS_XAW = 13  // adjoint, axis 0: w = D W', then D^T (lam, h J(w)^T lam / 6)
};

// Pointers of one pass; every field pointer addresses the concatenated field of all
// groups (the kernel adds the group offset).
struct PassArgs {
    float2* psi;              // single field: D1 in/out, FIRST in, LAST2/AF/D2U out, XAW in (lambda)
    float2* psi_out;          // LAST2: write psi' here instead of psi (a step out of place), or null
    float2* A;                // field pair in/out
    float2* B;
    const float2* aux0;       // extra inputs: XAW (W before its axis-0 propagator), AS (a, k1), AF (psi_n)
    const float2* aux1;
    double* vbar;             // FP64 potential-gradient accumulator (concatenated), XAW/AS/AF
    int adj;                  // apply the transpose of D
    int lines;                // tile schedule: lines (contiguous axis) or columns (strided) per
                              // workgroup, 0 = default
    int seq;                  // 0: fields transformed together; 1: one after the other (half the
                              // LDS); 2: as 1 with the second field loaded after the first;
                              // 3: one thread per field (twice the threads)
    int radix;                // values per thread in the transform: 16 (0 = default) or 8
    int f64;                  // transforms, propagator multiply and delta add in FP64 (radix 8)
    int occ;                  // minimum waves per SIMD the kernel is compiled for (0/1 = none, 4)
    int twice;                // D1: apply the half-step propagator twice (a whole step)
    int64_t step_off;
    const int64_t* step_base; // step = step_off (+ *step_base when not null)
};

// Arguments of the adaptive 1D integrator (k_line_ark45).
struct ArkArgs {
    double t_span;            // integrate every instance over [0, t_span]
    double tol;               // accept a step when its error estimate is at most tol
    double alpha, gamma;      // L(k) = -i alpha k^2 - gamma
    double kscale;            // 2 pi / (hi - lo): k_m = kscale * (m < n/2 ? m : m - n)
    int64_t max_attempts;     // trial steps per instance at most
    int64_t inst_base;        // plan-wide index of the group's first instance
    int64_t log_cap;          // entries per instance in h_log
    double* h;                // [ninst] in: first trial step; out: next trial step
    int64_t* stats;           // [ninst][3] accepted, rejected, reached t_span
    double* h_log;            // [ninst][log_cap] accepted step sizes, or null
    int explicit_L;           // 1: the explicit comparison method (no interaction picture)
};

// Constants of the final diagnostic sum (FP64).
struct DiagConst {
    double dV;
    double alpha;
    double half_g;
};

// Work list of a pass launched once over several groups (kernels_pass_merged.hip): the
// groups' kernel parameters live in device memory; workgroup b belongs to entry k with
// block0[k] <= b < block0[k + 1] (each entry starts on a multiple of 8 blocks) and runs
// tile b - block0[k] of its nblk[k].
constexpr int kMaxMerged = 64;
struct MergedList {
    const GroupDev* groups;  // device, every group of the plan in plan order
    int count;               // entries
    int gid[kMaxMerged];     // plan-order group of each entry
    uint32_t block0[kMaxMerged];
    uint32_t nblk[kMaxMerged];
};

int axis_lines(int N, int axis, int n0);
// Whether a (lines, seq) schedule of a pass is compiled for this length and axis.
bool axis_schedule_ok(int N, int mode, int axis, int n0, int lines, int seq, int radix, bool f64, int occ = 1);

hipError_t launch_axis(const GroupDev& g, int axis, int mode, const PassArgs& a, hipStream_t s);
// The merged pass: lengths 128 and 256, forward-step kinds (FIRST, D2, LF, XF, LAST2),
// FP32 transforms, 256-thread tiles of merged_tile_lines(N) lines or columns; smem =
// the largest merged_lds_bytes of its entries.
hipError_t launch_axis_merged(const MergedList& ml, int mode, int axis, bool noise, uint32_t blocks, size_t smem,
                              const PassArgs& a, hipStream_t s);
size_t merged_lds_bytes(int N, int mode, int axis);
int merged_tile_lines(int N);
hipError_t launch_axis_adjoint(const GroupDev& g, int axis, int mode, const PassArgs& a, hipStream_t s);
hipError_t launch_axis_d(const GroupDev& g, int axis, int mode, const PassArgs& a, hipStream_t s);
hipError_t launch_axis_first(const GroupDev& g, int axis, int mode, const PassArgs& a, hipStream_t s);
hipError_t launch_axis_xf(const GroupDev& g, int axis, const PassArgs& a, hipStream_t s);
hipError_t launch_axis_si(const GroupDev& g, int axis, const PassArgs& a, hipStream_t s);
hipError_t launch_axis_last(const GroupDev& g, int axis, int mode, const PassArgs& a, hipStream_t s);
hipError_t launch_line_adjoint(const GroupDev& g, const float2* psi_n, float2* lam, double* vbar, int64_t step,
                               const int64_t* step_base, hipStream_t s);
hipError_t launch_vbar_to_float(const double* vbar, float* out, int64_t n, hipStream_t s);
// io (groups with a k-space state buffer, GroupDev::K, only): bit 0 reads the state from K
// instead of transforming psi, bit 1 leaves it in K instead of transforming it back into psi.
// out: where the lines are written (null: back into psi).
hipError_t launch_line_step(const GroupDev& g, float2* psi, int nsteps, int64_t step_off, const int64_t* step_base, bool f64,
                            int radix, bool semi_implicit, hipStream_t s, int io = 0, float2* out = nullptr);
hipError_t launch_line_ark45(const GroupDev& g, float2* psi, const ArkArgs& x, hipStream_t s);
hipError_t launch_diag_axis(const GroupDev& g, int axis, const float2* psi, double kscale, double* part,
                            hipStream_t s);
hipError_t launch_diag_final(const GroupDev& g, const DiagConst& c, const double* p0, const double* p1,
                             const double* p2, double* out, int* flag, hipStream_t s);
hipError_t launch_overlap(const GroupDev& g, double dV, const float2* phi, const float2* psi, double* out,
                          hipStream_t s);
hipError_t launch_moments(const GroupDev& g, const float2* psi, double* mean, double* var, hipStream_t s);
hipError_t launch_counter(int64_t* c, int64_t v, int add, hipStream_t s);
hipError_t launch_philox(uint32_t k0, uint32_t k1, const uint32_t* ctr, int64_t n, uint32_t* out, hipStream_t s);
hipError_t launch_noise(const GroupDev& g, int64_t step, float2* xi, hipStream_t s);
hipError_t launch_fft_lines(const float2* in, float2* out, int64_t n, int64_t nlines, int sign, const float2* tw,
                            hipStream_t s);

}  // namespace rk4ip
