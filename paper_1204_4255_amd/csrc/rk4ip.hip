// rk4ip.hip -- host runtime of the RK4IP library: validation, plan-time tables,
// workspace carving, the per-step pass schedule, hipGraph replay, FP64 diagnostics and
// the C ABI declared in include/rk4ip.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/rk4ip.h"
#include "device_common.h"
#include "launch.h"

using rk4ip::GroupDev;

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr size_t kAlign = 256;
constexpr uint32_t kKnownFlags = RK4IP_FLAG_GRAPH | RK4IP_FLAG_AUTOTUNE | RK4IP_FLAG_FUSE_1D |
                                  RK4IP_FLAG_FP64_TRANSFORMS | RK4IP_FLAG_SEMI_IMPLICIT | RK4IP_FLAG_MERGE_GROUPS;
constexpr uint32_t kMaxNoiseSubsteps = 1024;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

// A cosine / sine group runs through the n-point transform of its reordered line (FP32
// transforms, no noise in the potential) or else through the even / odd extension of its
// half domain, twice the stored points (the FP64-transform form, and the line kernel
// variant that carries the potential's extra terms).
bool basis_ext(const rk4ip_problem& p, uint32_t flags) {
    return p.basis && ((flags & RK4IP_FLAG_FP64_TRANSFORMS) || p.sigma_V != 0.0);
}
bool basis_dct(const rk4ip_problem& p, uint32_t flags) { return p.basis && !basis_ext(p, flags); }

// Length of the transform along axis a.
int64_t transform_len(const rk4ip_problem& p, int a, uint32_t flags) {
    return (a == 0 && basis_ext(p, flags)) ? 2 * p.n[0] : p.n[a];
}

// The problem seen by the Fourier tables: for a group run on its extension, the
// extension's length and a domain twice as long (so k_m = pi m / L).
rk4ip_problem transform_problem(const rk4ip_problem& p, uint32_t flags) {
    rk4ip_problem q = p;
    if (basis_ext(p, flags)) {
        q.n[0] = 2 * p.n[0];
        q.hi[0] = p.hi[0] + (p.hi[0] - p.lo[0]);
    }
    return q;
}

// 1D groups that the k-space line step runs: Fourier basis, no extra potential terms,
// FP32 transforms. They keep their k-space state in the workspace between launches.
bool is_kline(const rk4ip_problem& p, uint32_t flags) {
    return p.ndim == 1 && !p.basis && !p.conv_K && p.sigma_V == 0.0 && !(flags & RK4IP_FLAG_FP64_TRANSFORMS);
}

int ilog2i(int64_t v) {
    int r = 0;
    while ((int64_t(1) << r) < v) r++;
    return r;
}

// Tile schedule of one pass (see PassArgs): lines or columns per workgroup, joint,
// sequential or split field transforms, values per thread in the transform.
struct Sched {
    int occ = 0;    // 4: the variant compiled for four waves per SIMD
    int lines = 0;
    int seq = 0;
    int radix = 0;
};

struct GroupHost {
    rk4ip_problem p;
    GroupDev d;
    int64_t M = 0;
    int64_t first_inst = 0;  // index of the group's first instance among all instances
    size_t tab_off[3] = {0, 0, 0};   // E table offsets in the workspace
    size_t tw_off[3] = {0, 0, 0};    // twiddle table offsets
    size_t tab64_off[3] = {0, 0, 0}; // FP64 copies (FP64-transform plans)
    size_t tw64_off[3] = {0, 0, 0};
    size_t part_off[3] = {0, 0, 0};  // diagnostic partials (batch * M/n_a * 4 doubles)
    size_t conv_off = 0;             // transform of the non-local kernel (1D groups with one)
    size_t e2_off = 0;               // (e^{L h} - 1)/n of a 1D Fourier group (its k-space line step)
    size_t k_off = 0;                // k-space state of a group run by the k-space line step
    bool kline = false;              // run by the k-space line step (state in the workspace)
    bool dct = false;                // cosine / sine group run through its reordered n-point transform
    double dV = 1.0;
};

// Workspace layout computed identically by rk4ip_workspace_bytes and rk4ip_plan.
struct Layout {
    size_t gdev = 0;     // the groups' kernel parameters (merged launches)
    size_t header = 0;   // step counter + sticky flag
    size_t fields = 0;   // A and B
    size_t total = 0;
    int64_t points = 0;
};

int validate(const rk4ip_problem* probs, int nprob, uint32_t flags) {
    if (!probs || nprob < 1 || nprob > 4096) return RK4IP_ERR_INVALID_ARG;
    if (flags & ~kKnownFlags) return RK4IP_ERR_INVALID_ARG;
    const double dt0 = probs[0].dt;
    int64_t ninst = 0;
    for (int i = 0; i < nprob; i++) {
        const rk4ip_problem& p = probs[i];
        if (p.basis < 0 || p.basis > 2) return RK4IP_ERR_INVALID_ARG;
        // the cosine and sine bases: 1D half domains, local potential
        if (p.basis && (p.ndim != 1 || p.conv_K)) return RK4IP_ERR_UNSUPPORTED_SHAPE;
        if (p.noise_substeps > kMaxNoiseSubsteps || (p.noise_substeps > 1 && !is_pow2(p.noise_substeps)))
            return RK4IP_ERR_INVALID_ARG;
        if (!(p.dt > 0.0) || !std::isfinite(p.dt) || p.dt != dt0) return RK4IP_ERR_INVALID_ARG;
        if (!std::isfinite(p.alpha) || !std::isfinite(p.gamma) || p.gamma < 0.0) return RK4IP_ERR_INVALID_ARG;
        if (!std::isfinite(p.g_nl) || !std::isfinite(p.sigma) || p.sigma < 0.0) return RK4IP_ERR_INVALID_ARG;
        if (!std::isfinite(p.sigma_V) || p.sigma_V < 0.0) return RK4IP_ERR_INVALID_ARG;
        // the non-local potential is built for 1D groups
        if (p.conv_K && p.ndim != 1) return RK4IP_ERR_UNSUPPORTED_SHAPE;
        if (p.conv_K && p.ndim == 1 && p.n[0] >= 1 && p.n[0] <= 4096) {
            for (int64_t d = 0; d < p.n[0]; d++)
                if (!std::isfinite(p.conv_K[d])) return RK4IP_ERR_INVALID_ARG;
        }
        if (p.batch < 1 || p.batch > (int64_t(1) << 31)) return RK4IP_ERR_INVALID_ARG;
        if ((uint64_t)p.id_base + (uint64_t)p.batch - 1 > 0xFFFFFFFFull) return RK4IP_ERR_INVALID_ARG;
        if (p.ndim < 1 || p.ndim > 3) return RK4IP_ERR_UNSUPPORTED_SHAPE;
        // FP64 transforms keep their tables and exchange buffers in LDS up to 2048 points
        const int64_t nmax = p.ndim == 1 ? ((flags & RK4IP_FLAG_FP64_TRANSFORMS) ? 2048 : 4096) : 1024;
        int64_t M = 1;
        for (int a = 0; a < 3; a++) {
            if (a < p.ndim) {
                if (!is_pow2(p.n[a]) || p.n[a] < 8 || transform_len(p, a, flags) > nmax) return RK4IP_ERR_UNSUPPORTED_SHAPE;
                if (!(p.hi[a] > p.lo[a]) || !std::isfinite(p.hi[a]) || !std::isfinite(p.lo[a]))
                    return RK4IP_ERR_INVALID_ARG;
                if (!std::isfinite(p.trap[a])) return RK4IP_ERR_INVALID_ARG;
                M *= p.n[a];
            } else if (p.n[a] != 1) {
                return RK4IP_ERR_UNSUPPORTED_SHAPE;
            }
        }
        // the pass kernels address a tile with 32-bit byte offsets from the instance origin,
        // so one instance must span less than 4 GiB of complex64 (M <= 2^29)
        if (M > (int64_t(1) << 29) || p.batch * M > (int64_t(1) << 40)) return RK4IP_ERR_UNSUPPORTED_SHAPE;
        ninst += p.batch;
    }
    if (ninst > (int64_t(1) << 31)) return RK4IP_ERR_INVALID_ARG;
    if (flags & RK4IP_FLAG_MERGE_GROUPS) {
        // the merged launches: RK4IP with FP32 transforms, lengths 128 and 256, tiles of
        // 2048/n columns on the strided axes
        if (flags & (RK4IP_FLAG_SEMI_IMPLICIT | RK4IP_FLAG_FP64_TRANSFORMS)) return RK4IP_ERR_UNSUPPORTED_SHAPE;
        if (nprob > rk4ip::kMaxMerged) return RK4IP_ERR_UNSUPPORTED_SHAPE;
        for (int i = 0; i < nprob; i++) {
            const rk4ip_problem& p = probs[i];
            if (p.ndim == 1) continue;
            for (int a = 0; a < p.ndim; a++) {
                if (p.n[a] != 128 && p.n[a] != 256) return RK4IP_ERR_UNSUPPORTED_SHAPE;
                if (a > 0 && p.n[0] < 2048 / p.n[a]) return RK4IP_ERR_UNSUPPORTED_SHAPE;
            }
        }
    }
    return RK4IP_OK;
}

// Offsets of every table and buffer; fills `gh` when non-null.
Layout layout(const rk4ip_problem* probs, int nprob, uint32_t flags, GroupHost* gh) {
    Layout L;
    size_t off = 0;
    L.header = off;
    off += kAlign;
    const bool f64 = (flags & RK4IP_FLAG_FP64_TRANSFORMS) != 0;
    for (int i = 0; i < nprob; i++) {
        const rk4ip_problem& p = probs[i];
        for (int a = 0; a < p.ndim; a++) {
            size_t e = off;
            off = align_up(off + sizeof(float2) * (size_t)transform_len(p, a, flags));
            size_t t = off;
            off = align_up(off + sizeof(float2) * (size_t)transform_len(p, a, flags));
            size_t e64 = 0, t64 = 0;
            if (f64) {
                e64 = off;
                off = align_up(off + sizeof(double2) * (size_t)transform_len(p, a, flags));
                t64 = off;
                off = align_up(off + sizeof(double2) * (size_t)transform_len(p, a, flags));
            }
            if (gh) {
                gh[i].tab_off[a] = e;
                gh[i].tw_off[a] = t;
                gh[i].tab64_off[a] = e64;
                gh[i].tw64_off[a] = t64;
            }
        }
    }
    for (int i = 0; i < nprob; i++) {
        const rk4ip_problem& p = probs[i];
        if (p.conv_K) {
            if (gh) gh[i].conv_off = off;
            off = align_up(off + sizeof(float2) * (size_t)p.n[0]);
        }
        if (is_kline(p, flags)) {
            // (e^{L h} - 1)/n of a k-space line
            if (gh) gh[i].e2_off = off;
            off = align_up(off + sizeof(float2) * (size_t)p.n[0]);
        }
        if (basis_dct(p, flags)) {
            // the two FP64 mode-pairing tables of a cosine / sine line
            if (gh) {
                gh[i].e2_off = off;
                gh[i].dct = true;
            }
            off = align_up(off + 2 * sizeof(double2) * (size_t)p.n[0]);
        }
    }
    for (int i = 0; i < nprob; i++) {
        const rk4ip_problem& p = probs[i];
        if (is_kline(p, flags)) {
            if (gh) {
                gh[i].k_off = off;
                gh[i].kline = true;
            }
            off = align_up(off + sizeof(float2) * (size_t)(p.batch * p.n[0]));
        }
    }
    for (int i = 0; i < nprob; i++) {
        const rk4ip_problem& p = probs[i];
        int64_t M = p.n[0] * p.n[1] * p.n[2];
        for (int a = 0; a < p.ndim; a++) {
            if (gh) gh[i].part_off[a] = off;
            off = align_up(off + sizeof(double) * 4 * (size_t)(p.batch * (M / p.n[a])));
        }
        L.points += p.batch * M;
    }
    if (flags & RK4IP_FLAG_MERGE_GROUPS) {
        L.gdev = off;
        off = align_up(off + sizeof(GroupDev) * (size_t)nprob);
    }
    L.fields = off;
    off = align_up(off + 2 * sizeof(float2) * (size_t)L.points);
    L.total = off;
    return L;
}

// Per-group kernel parameters and table pointers into the workspace `ws` (the offsets come
// from layout); the group's field starts at point `offset` of the concatenated field. The
// tables themselves are written by the caller.
void fill_group(GroupHost& g, char* ws, uint32_t flags, int64_t offset) {
    const bool f64 = (flags & RK4IP_FLAG_FP64_TRANSFORMS) != 0;
    const rk4ip_problem& p = g.p;
    GroupDev& d = g.d;
    std::memset(&d, 0, sizeof(d));
    d.ndim = p.ndim;
    g.M = 1;
    g.dV = 1.0;
    for (int a = 0; a < 3; a++) {
        const int64_t nt = transform_len(p, a, flags);
        d.n[a] = (int)nt;
        d.log2n[a] = ilog2i(nt);
        g.M *= p.n[a];
        if (a < p.ndim) {
            const double dx = (p.hi[a] - p.lo[a]) / (double)p.n[a];
            g.dV *= dx;
            // a cosine / sine group's points are the cell centres lo + (j + 1/2) dx
            d.lo[a] = (float)(p.basis ? p.lo[a] + 0.5 * dx : p.lo[a]);
            d.dx[a] = (float)dx;
            d.half_trap[a] = (float)(0.5 * p.trap[a]);
            d.inv_n[a] = (float)(1.0 / (double)nt);
        }
    }
    d.basis = p.basis;
    d.M = g.M;
    d.batch = p.batch;
    d.offset = offset;
    d.h = (float)p.dt;
    d.gnl = (float)p.g_nl;
    d.noise_c = (float)(p.dt * p.sigma / std::sqrt(2.0 * p.dt * g.dV));
    d.xi_scale = (float)(1.0 / std::sqrt(2.0 * p.dt * g.dV));
    d.seed_lo = (uint32_t)(p.seed & 0xFFFFFFFFu);
    d.seed_hi = (uint32_t)(p.seed >> 32);
    d.id_base = p.id_base;
    d.has_noise = (p.sigma != 0.0 || p.sigma_V != 0.0) ? 1 : 0;
    d.has_vnoise = p.sigma_V != 0.0 ? 1 : 0;
    d.vnoise_c = (float)(p.sigma_V / std::sqrt(p.dt * g.dV));
    d.noise_sub = p.noise_substeps > 1 ? (int)p.noise_substeps : 1;
    d.inv_sqrt_sub = (float)(1.0 / std::sqrt((double)d.noise_sub));  // a power of two or its root
    d.Vgrid = p.V_grid;
    for (int a = 0; a < p.ndim; a++) {
        d.E[a] = reinterpret_cast<const float2*>(ws + g.tab_off[a]);
        d.tw[a] = reinterpret_cast<const float2*>(ws + g.tw_off[a]);
        if (f64) {
            d.E64[a] = reinterpret_cast<const double2*>(ws + g.tab64_off[a]);
            d.tw64[a] = reinterpret_cast<const double2*>(ws + g.tw64_off[a]);
        }
    }
    if (g.kline) d.E2 = reinterpret_cast<const float2*>(ws + g.e2_off);
    if (g.dct) {
        d.pairT1 = reinterpret_cast<const double2*>(ws + g.e2_off);
        d.pairT2 = d.pairT1 + p.n[0];
    }
    if (g.kline) d.K = reinterpret_cast<float2*>(ws + g.k_off);
    if (p.conv_K) d.convK = reinterpret_cast<const float2*>(ws + g.conv_off);
}

}  // namespace

struct rk4ip_plan_s {
    std::vector<GroupHost> groups;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    uint32_t flags = 0;
    int device = 0;
    int64_t points = 0;
    int64_t ninst = 0;
    float2* A = nullptr;
    float2* B = nullptr;
    int64_t* counter = nullptr;
    int* flag = nullptr;
    bool f64 = false;  // FP64 transforms in the forward step
    bool si = false;   // the semi-implicit integrator in place of RK4
    // merged launches (RK4IP_FLAG_MERGE_GROUPS): one work list per (dimensionality, pass)
    struct Merged {
        int ndim, pass, mode, axis, role, twice;
        bool noise;
        uint32_t blocks;
        size_t smem;
        rk4ip::MergedList list;
    };
    std::vector<Merged> merged;
    std::string err;
    std::vector<std::vector<std::string>> sched_names;  // [group][pass]
    std::vector<std::vector<Sched>> sched;  // [group][pass]; zeros = default schedule
    // cached graphs of 1, 2, 4, ..., 32 steady-state steps on `graph_psi` (recorded when a
    // run first needs them)
    hipGraphExec_t graph[6] = {};
    hipGraph_t graph_src[6] = {};
    void* graph_psi = nullptr;
    hipStream_t capture_stream = nullptr;  // private stream the graph is recorded on
    // graphs of one adjoint segment (recompute, backward walk) for the buffers they were
    // recorded on
    hipGraphExec_t adj_fwd = nullptr, adj_bwd = nullptr;
    const void* adj_key[3] = {nullptr, nullptr, nullptr};  // store, lambda, vbar
    int64_t adj_M = 0;
    int sticky = RK4IP_OK;
    // per-pass event timing
    bool profiling = false;
    struct Timed {
        int group, pass;
        hipEvent_t a, b;
    };
    std::vector<Timed> timed;
    std::vector<hipEvent_t> spare;
    std::vector<std::vector<double>> prof_ms;     // [group][pass] summed ms
    std::vector<std::vector<int64_t>> prof_n;     // [group][pass] launches
};

namespace {

int fail(rk4ip_plan_t plan, int code, const std::string& msg) {
    if (plan) plan->err = msg;
    return code;
}

int fail_hip(rk4ip_plan_t plan, hipError_t e, const char* what) {
    if (plan) {
        plan->err = std::string(what) + ": " + hipGetErrorString(e);
        plan->sticky = RK4IP_ERR_HIP;
    }
    return RK4IP_ERR_HIP;
}

#define HIPCHK(plan, expr)                                           \
    do {                                                             \
        hipError_t e_ = (expr);                                      \
        if (e_ != hipSuccess) return fail_hip((plan), e_, #expr);    \
    } while (0)

void drop_step_graphs(rk4ip_plan_t plan) {
    for (int i = 0; i < 6; i++) {
        if (plan->graph[i]) (void)hipGraphExecDestroy(plan->graph[i]);
        if (plan->graph_src[i]) (void)hipGraphDestroy(plan->graph_src[i]);
        plan->graph[i] = nullptr;
        plan->graph_src[i] = nullptr;
    }
    plan->graph_psi = nullptr;
}

void drop_graph(rk4ip_plan_t plan) {
    drop_step_graphs(plan);
    if (plan->adj_fwd) (void)hipGraphExecDestroy(plan->adj_fwd);
    if (plan->adj_bwd) (void)hipGraphExecDestroy(plan->adj_bwd);
    plan->adj_fwd = plan->adj_bwd = nullptr;
    plan->adj_M = 0;
}

// Waits for the plan's stream, frees the HIP objects the plan created (graph, capture
// stream, timing events) and the plan itself. The workspace is the caller's.
void release_plan(rk4ip_plan_t plan) {
    (void)hipStreamSynchronize(plan->stream);
    drop_graph(plan);
    if (plan->capture_stream) (void)hipStreamDestroy(plan->capture_stream);
    for (auto& t : plan->timed) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    for (auto e : plan->spare) (void)hipEventDestroy(e);
    delete plan;
}

// Tables of one axis (FP64 arithmetic; stored in FP32, and in FP64 for FP64-transform plans).
void build_tables(const rk4ip_problem& p, int a, std::vector<float2>& E, std::vector<float2>& tw,
                  std::vector<double2>* E64 = nullptr, std::vector<double2>* tw64 = nullptr,
                  std::vector<float2>* E2 = nullptr) {
    const int64_t n = p.n[a];
    const double Lx = p.hi[a] - p.lo[a];
    const double h = p.dt;
    const double damp = (a == 0) ? std::exp(-p.gamma * h / 2.0) : 1.0;
    const double em1 = (a == 0) ? std::expm1(-p.gamma * h / 2.0) : 0.0;
    E.resize(n);
    tw.resize(n);
    if (E64) E64->resize(n);
    if (tw64) tw64->resize(n);
    if (E2) E2->resize(n);
    const double inv_n = 1.0 / (double)n;  // exact power of two
    for (int64_t m = 0; m < n; m++) {
        const double k = 2.0 * kPi / Lx * (double)(m < n / 2 ? m : m - n);
        const double theta = p.alpha * k * k * h / 2.0;
        const double sh = std::sin(theta / 2.0);
        // E - 1 = damp cos(theta) - 1 - i damp sin(theta), with
        // damp cos(theta) - 1 = (damp - 1) - 2 damp sin^2(theta/2) (no cancellation)
        const double c = em1 - 2.0 * damp * sh * sh;
        const double s = -damp * std::sin(theta);
        E[m] = make_float2((float)(c * inv_n), (float)(s * inv_n));
        const double ang = 2.0 * kPi * (double)m / (double)n;
        tw[m] = make_float2((float)std::cos(ang), (float)-std::sin(ang));
        if (E64) (*E64)[m] = make_double2(c * inv_n, s * inv_n);
        if (E2) {
            // e^{L h} - 1 = damp^2 e^{-2 i theta} - 1, written without cancellation:
            // damp^2 cos(2 theta) - 1 = (damp^2 - 1) - 2 damp^2 sin^2(theta)
            const double d2 = damp * damp, em2 = std::expm1(-p.gamma * h), st = std::sin(theta);
            const double c2 = (a == 0 ? em2 : 0.0) - 2.0 * d2 * st * st;
            const double s2 = -d2 * std::sin(2.0 * theta);
            (*E2)[m] = make_float2((float)(c2 * inv_n), (float)(s2 * inv_n));
        }
        if (tw64) (*tw64)[m] = make_double2(std::cos(ang), -std::sin(ang));
    }
}

// Transform of the non-local kernel times dV/n (FP64 sums over a twiddle table, stored
// FP32): kh_m = (dV/n) sum_d K[d] e^{-2 pi i m d / n}.
void build_conv_table(const rk4ip_problem& p, double dV, std::vector<float2>& kh) {
    const int64_t n = p.n[0];
    std::vector<double> c(n), sn(n);
    for (int64_t q = 0; q < n; q++) {
        c[q] = std::cos(2.0 * kPi * (double)q / (double)n);
        sn[q] = std::sin(2.0 * kPi * (double)q / (double)n);
    }
    kh.resize(n);
    for (int64_t m = 0; m < n; m++) {
        double re = 0.0, im = 0.0;
        for (int64_t d = 0; d < n; d++) {
            const int64_t q = (m * d) & (n - 1);
            re += p.conv_K[d] * c[q];
            im -= p.conv_K[d] * sn[q];
        }
        kh[m] = make_float2((float)(re * dV / (double)n), (float)(im * dV / (double)n));
    }
}

// Tables of a cosine / sine line run through its reordered n-point transform (FP64
// arithmetic, stored FP32). The line v_e = s_e f_{j(e)}, with j(e) = 2e for e < n/2 and
// 2(n - 1 - e) + 1 above, s_e = -1 on the odd points in the sine basis, has V = F v with
// cosine coefficients X_m = (W^m V_m + W^-m V_{n-m})/2, W = e^{-i pi/(2n)} (Makhoul's
// algorithm). e^{L h/2} multiplies cosine coefficient m by E_m, which maps V to
// A_m V_m + B_m V_{n-m} with A_m = (E_m + E_{n-m})/2, B_m = (E_m - E_{n-m}) e^{i pi m/n}/2
// (A_0 = E_0, B_0 = 0). Cosine basis: E_m at k = pi m/L. Sine basis: the cosine coefficient m
// of the sign-alternated line is the sine coefficient n - 1 - m, at k = pi (n - m)/L.
// Stored: T1 = (A - 1)/n (without cancellation, from the expm1 form of E - 1), the FFT
// twiddles, T2 = B/n. T1 and T2 stay in FP64: each pairs a low mode with a high one through
// factors of order one whose sum nearly cancels, so their rounding would reach the field at
// the size of the field, the same every step.
void build_basis_tables(const rk4ip_problem& p, std::vector<double2>& T12, std::vector<float2>& tw) {
    const int64_t n = p.n[0];
    const double L = p.hi[0] - p.lo[0], h = p.dt;
    const double damp = std::exp(-p.gamma * h / 2.0), em1 = std::expm1(-p.gamma * h / 2.0);
    auto em1_of = [&](int64_t m, double& c, double& s) {  // E_m - 1
        const double k = kPi / L * (double)(p.basis == 1 ? m : n - m);
        const double theta = p.alpha * k * k * h / 2.0;
        const double sh = std::sin(theta / 2.0);
        c = em1 - 2.0 * damp * sh * sh;
        s = -damp * std::sin(theta);
    };
    T12.resize(2 * n);  // T1 then T2
    tw.resize(n);
    const double inv_n = 1.0 / (double)n;
    for (int64_t m = 0; m < n; m++) {
        double ac, as;
        em1_of(m, ac, as);
        if (m == 0) {
            T12[m] = make_double2(ac * inv_n, as * inv_n);
            T12[n + m] = make_double2(0.0, 0.0);
        } else {
            double bc, bs;
            em1_of(n - m, bc, bs);
            const double dc = 0.5 * (ac - bc), ds = 0.5 * (as - bs);  // (E_m - E_{n-m})/2
            const double ph = kPi * (double)m / (double)n;
            const double cp = std::cos(ph), sp = std::sin(ph);
            T12[m] = make_double2(0.5 * (ac + bc) * inv_n, 0.5 * (as + bs) * inv_n);
            T12[n + m] = make_double2((dc * cp - ds * sp) * inv_n, (dc * sp + ds * cp) * inv_n);
        }
        const double ang = 2.0 * kPi * (double)m / (double)n;
        tw[m] = make_float2((float)std::cos(ang), (float)-std::sin(ang));
    }
}

// The passes of a 2D/3D group. A run of steps is OPEN (at its first step), then for every
// step but the last the MID passes and the NEXT pass (which ends the step and opens the
// following one), and for the last step the MID passes and CLOSE.
enum Role { ROLE_OPEN, ROLE_MID, ROLE_NEXT, ROLE_CLOSE };
struct PassDef {
    int axis, mode, role;
    int twice = 0;  // D1 on axis 0 applied twice: the end of one step and the start of the next
};

int pass_list(int ndim, bool si, PassDef* out) {
    if (si) {
        // in place on psi: D_0, the middle axes, the midpoint iteration between the two
        // half steps of the last axis, the middle axes again, then D_0 twice where two
        // steps meet (in one pass) or once at the end of the run
        const int last = ndim - 1;
        int k = 0;
        out[k++] = {0, rk4ip::PASS_D1, ROLE_OPEN};
        for (int a = 1; a < last; a++) out[k++] = {a, rk4ip::PASS_D1, ROLE_MID};
        out[k++] = {last, rk4ip::PASS_SI, ROLE_MID};
        for (int a = last - 1; a >= 1; a--) out[k++] = {a, rk4ip::PASS_D1, ROLE_MID};
        out[k++] = {0, rk4ip::PASS_D1, ROLE_NEXT, 1};
        out[k++] = {0, rk4ip::PASS_D1, ROLE_CLOSE};
        return k;
    }
    if (ndim == 2) {
        const PassDef seq[4] = {{0, rk4ip::PASS_FIRST, ROLE_OPEN},
                                {1, rk4ip::PASS_LF, ROLE_MID},
                                {0, rk4ip::PASS_XF, ROLE_NEXT},
                                {0, rk4ip::PASS_LAST2, ROLE_CLOSE}};
        for (int i = 0; i < 4; i++) out[i] = seq[i];
        return 4;
    }
    const PassDef seq[6] = {{0, rk4ip::PASS_FIRST, ROLE_OPEN}, {1, rk4ip::PASS_D2, ROLE_MID},
                            {2, rk4ip::PASS_LF, ROLE_MID},     {1, rk4ip::PASS_D2, ROLE_MID},
                            {0, rk4ip::PASS_XF, ROLE_NEXT},    {0, rk4ip::PASS_LAST2, ROLE_CLOSE}};
    for (int i = 0; i < 6; i++) out[i] = seq[i];
    return 6;
}
constexpr int kMaxPasses = 6;

const char* mode_name(int mode) {
    switch (mode) {
        case rk4ip::PASS_D1: return "D1";
        case rk4ip::PASS_D2: return "D2";
        case rk4ip::PASS_FIRST: return "FIRST";
        case rk4ip::PASS_LAST2: return "LAST2";
        case rk4ip::PASS_LF: return "LF";
        case rk4ip::PASS_XF: return "XF";
        case rk4ip::PASS_SI: return "SI";
        default: return "?";
    }
}

hipEvent_t take_event(rk4ip_plan_t plan) {
    if (!plan->spare.empty()) {
        hipEvent_t e = plan->spare.back();
        plan->spare.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Run `launch` bracketed by an event pair when profiling (never inside a capture).
template <class F>
int timed_launch(rk4ip_plan_t plan, hipStream_t stream, int group, int pass, bool capturing, F&& launch) {
    if (!plan->profiling || capturing) {
        HIPCHK(plan, launch());
        return RK4IP_OK;
    }
    hipEvent_t a = take_event(plan), b = take_event(plan);
    if (!a || !b) return fail(plan, RK4IP_ERR_HIP, "hipEventCreate failed");
    HIPCHK(plan, hipEventRecord(a, stream));
    HIPCHK(plan, launch());
    HIPCHK(plan, hipEventRecord(b, stream));
    plan->timed.push_back({group, pass, a, b});
    return RK4IP_OK;
}

// Fold recorded event pairs into the per-pass sums (waits for them).
int collect_profile(rk4ip_plan_t plan) {
    for (auto& t : plan->timed) {
        HIPCHK(plan, hipEventSynchronize(t.b));
        float ms = 0.f;
        HIPCHK(plan, hipEventElapsedTime(&ms, t.a, t.b));
        plan->prof_ms[t.group][t.pass] += ms;
        plan->prof_n[t.group][t.pass] += 1;
        plan->spare.push_back(t.a);
        plan->spare.push_back(t.b);
    }
    plan->timed.clear();
    return RK4IP_OK;
}

// Mean time (ms) of `reps` launches of one pass with a given schedule, on the work fields.
int time_pass(rk4ip_plan_t plan, const GroupHost& g, const PassDef& def, const Sched& sc, int reps, float* ms) {
    const int axis = def.axis, mode = def.mode;
    rk4ip::PassArgs pa{};
    pa.A = plan->A;
    pa.B = plan->B;
    pa.psi = (mode == rk4ip::PASS_FIRST) ? plan->B : plan->A;  // same tiles are read before written
    pa.twice = def.twice;
    pa.step_off = 1;
    pa.f64 = plan->f64 ? 1 : 0;
    pa.lines = sc.lines;
    pa.seq = sc.seq;
    pa.radix = sc.radix;
    pa.occ = sc.occ;
    hipStream_t st = plan->stream;
    for (int i = 0; i < 2; i++) HIPCHK(plan, rk4ip::launch_axis(g.d, axis, mode, pa, st));
    hipEvent_t a = take_event(plan), b = take_event(plan);
    if (!a || !b) return fail(plan, RK4IP_ERR_HIP, "hipEventCreate failed");
    HIPCHK(plan, hipEventRecord(a, st));
    for (int i = 0; i < reps; i++) HIPCHK(plan, rk4ip::launch_axis(g.d, axis, mode, pa, st));
    HIPCHK(plan, hipEventRecord(b, st));
    HIPCHK(plan, hipEventSynchronize(b));
    HIPCHK(plan, hipEventElapsedTime(ms, a, b));
    *ms /= (float)reps;
    plan->spare.push_back(a);
    plan->spare.push_back(b);
    return RK4IP_OK;
}

// Mean time (ms) of `reps` launches of eight 1D steps with `rr` values per thread, on the
// work field A (its contents are irrelevant; a k-space line keeps its state in the
// workspace, as in the steady state of a run).
int time_line(rk4ip_plan_t plan, const GroupHost& g, int rr, int reps, float* ms) {
    hipStream_t st = plan->stream;
    const int io = g.kline ? 3 : 0;
    if (g.kline) HIPCHK(plan, rk4ip::launch_line_step(g.d, plan->A, 0, 1, nullptr, false, rr, plan->si, st, 2));
    for (int i = 0; i < 2; i++)
        HIPCHK(plan, rk4ip::launch_line_step(g.d, plan->A, 8, 1, nullptr, false, rr, plan->si, st, io));
    hipEvent_t a = take_event(plan), b = take_event(plan);
    if (!a || !b) return fail(plan, RK4IP_ERR_HIP, "hipEventCreate failed");
    HIPCHK(plan, hipEventRecord(a, st));
    for (int i = 0; i < reps; i++)
        HIPCHK(plan, rk4ip::launch_line_step(g.d, plan->A, 8, 1, nullptr, false, rr, plan->si, st, io));
    HIPCHK(plan, hipEventRecord(b, st));
    HIPCHK(plan, hipEventSynchronize(b));
    HIPCHK(plan, hipEventElapsedTime(ms, a, b));
    *ms /= (float)reps;
    plan->spare.push_back(a);
    plan->spare.push_back(b);
    return RK4IP_OK;
}

// Tuning cache: a flat JSON object {"key": [lines, seq], ...} in the file named by
// RK4IP_TUNE_CACHE (optional).
std::string tune_key(const GroupHost& g, int pass, bool si) {
    char k[160];
    std::snprintf(k, sizeof(k), "gfx950|n=%lld,%lld,%lld|b=%lld|pass=%d%s%s", (long long)g.p.n[0],
                  (long long)g.p.n[1], (long long)g.p.n[2], (long long)g.p.batch, pass, g.d.E64[0] ? "|f64" : "",
                  si ? "|si" : "");
    return k;
}

bool cache_lookup(const std::string& text, const std::string& key, Sched* sc) {
    const std::string q = "\"" + key + "\"";
    size_t p = text.find(q);
    if (p == std::string::npos) return false;
    p = text.find('[', p);
    if (p == std::string::npos) return false;
    // [lines, seq, radix] or [lines, seq, radix, occ]
    sc->occ = 0;
    const int n = std::sscanf(text.c_str() + p, "[ %d , %d , %d , %d ]", &sc->lines, &sc->seq, &sc->radix, &sc->occ);
    return n >= 3;
}

// The schedule an FP64-transform pass runs without tuning: the first compiled one in a
// fixed order of preference (half the default lines on the contiguous axis, the default
// columns on a strided one; both fields at once before one after the other).
bool default_f64_sched(const GroupHost& g, int axis, int mode, Sched* out) {
    const int N = (int)g.p.n[axis], n0 = (int)g.p.n[0];
    const int cl = rk4ip::axis_lines(N, 0, n0);
    const int contig_pref[] = {cl / 2, cl / 4, cl, 1};
    const int strided_pref[] = {rk4ip::axis_lines(N, axis, n0), 8, 4, 16};
    for (int i = 0; i < 4; i++) {
        const int lines = axis == 0 ? contig_pref[i] : strided_pref[i];
        if (lines < 1) continue;
        for (int sq = 0; sq < 3; sq++) {
            if (rk4ip::axis_schedule_ok(N, mode, axis, n0, lines, sq, 8, true)) {
                out->lines = lines;
                out->seq = sq;
                out->radix = 8;
                return true;
            }
        }
    }
    return false;
}

// Work lists of the merged launches (RK4IP_FLAG_MERGE_GROUPS): for every dimensionality
// present and every pass of its list, the groups of that dimensionality in plan order, each
// starting on a multiple of 8 workgroups (so the XCD-aware tile order of a group is the
// one it has alone). The groups' kernel parameters are uploaded to the workspace at
// `gdev`. Every group's schedule is set to the merged one (radix 8, 256 threads).
int build_merged(rk4ip_plan_t plan, size_t gdev) {
    const int ng = (int)plan->groups.size();
    std::vector<GroupDev> devs(ng);
    for (int i = 0; i < ng; i++) devs[i] = plan->groups[i].d;
    GroupDev* dptr = reinterpret_cast<GroupDev*>(plan->ws + gdev);
    HIPCHK(plan, hipMemcpy(dptr, devs.data(), sizeof(GroupDev) * (size_t)ng, hipMemcpyHostToDevice));
    for (int nd = 2; nd <= 3; nd++) {
        std::vector<int> members;
        for (int i = 0; i < ng; i++)
            if (plan->groups[i].p.ndim == nd) members.push_back(i);
        if (members.empty()) continue;
        PassDef defs[kMaxPasses];
        const int np = pass_list(nd, false, defs);
        for (int k = 0; k < np; k++) {
            rk4ip_plan_s::Merged m{};
            m.ndim = nd;
            m.pass = k;
            m.mode = defs[k].mode;
            m.axis = defs[k].axis;
            m.role = defs[k].role;
            m.twice = defs[k].twice;
            m.list.groups = dptr;
            m.list.count = (int)members.size();
            uint32_t b0 = 0;
            for (size_t e = 0; e < members.size(); e++) {
                GroupHost& g = plan->groups[members[e]];
                const int N = (int)g.p.n[m.axis];
                const int lines = rk4ip::merged_tile_lines(N);
                const int64_t nl = g.p.batch * (g.M / g.p.n[m.axis]);  // lines along the axis
                const int64_t nb = (nl + lines - 1) / lines;
                if (nb > 0x7fffffffLL - b0) return fail(plan, RK4IP_ERR_UNSUPPORTED_SHAPE, "merged launch too large");
                m.list.gid[e] = members[e];
                m.list.block0[e] = b0;
                m.list.nblk[e] = (uint32_t)nb;
                b0 += (uint32_t)((nb + 7) / 8 * 8);
                m.noise = m.noise || g.d.has_noise;
                m.smem = std::max(m.smem, rk4ip::merged_lds_bytes(N, m.mode, m.axis));
                Sched sc;
                sc.lines = lines;
                sc.seq = 0;
                sc.radix = 8;
                plan->sched[members[e]][k] = sc;
            }
            m.blocks = b0;
            if (m.smem == 0) return fail(plan, RK4IP_ERR_UNSUPPORTED_SHAPE, "no merged kernel for this pass");
            plan->merged.push_back(m);
        }
    }
    return RK4IP_OK;
}

// Choose the fastest compiled schedule of every pass (RK4IP_FLAG_AUTOTUNE).
int autotune(rk4ip_plan_t plan) {
    const char* path = std::getenv("RK4IP_TUNE_CACHE");
    std::string text;
    if (path) {
        if (FILE* fh = std::fopen(path, "r")) {
            char buf[4096];
            size_t n;
            while ((n = std::fread(buf, 1, sizeof(buf), fh)) > 0) text.append(buf, n);
            std::fclose(fh);
        }
    }
    std::vector<std::pair<std::string, Sched>> fresh;
    HIPCHK(plan, hipMemsetAsync(plan->A, 0, 2 * sizeof(float2) * (size_t)plan->points, plan->stream));
    for (size_t gi = 0; gi < plan->groups.size(); gi++) {
        const GroupHost& g = plan->groups[gi];
        if (g.p.ndim == 1) {
            // the whole-line step: 16 or 8 values per thread (FP64 transforms use 8)
            if (plan->f64) continue;
            Sched c;
            if (cache_lookup(text, tune_key(g, 0, plan->si), &c) && (c.radix == 8 || c.radix == 16)) {
                plan->sched[gi][0] = c;
                continue;
            }
            float best = 1e30f;
            Sched pick;
            for (int rr : {16, 8}) {
                float ms = 0.f;
                int rc = time_line(plan, g, rr, 5, &ms);
                if (rc) return rc;
                if (ms < best) {
                    best = ms;
                    pick = Sched{};
                    pick.radix = rr;
                }
            }
            plan->sched[gi][0] = pick;
            fresh.push_back({tune_key(g, 0, plan->si), pick});
            continue;
        }
        if (!plan->merged.empty()) continue;  // the merged launches have one fixed schedule
        PassDef defs[kMaxPasses];
        const int np = pass_list(g.p.ndim, plan->si, defs);
        for (int i = 0; i < np; i++) {
            const int axis = defs[i].axis, mode = defs[i].mode;
            const int N = (int)g.p.n[axis], n0 = (int)g.p.n[0];
            Sched c;
            if (cache_lookup(text, tune_key(g, i, plan->si), &c) &&
                rk4ip::axis_schedule_ok(N, mode, axis, n0, c.lines, c.seq, c.radix, plan->f64, c.occ ? c.occ : 1)) {
                plan->sched[gi][i] = c;
                continue;
            }
            float best = 1e30f;
            Sched pick;
            const int cand_lines[] = {1, 2, 4, 8, 16, 32, 64, 128, 256};
            const int cand_radix[] = {16, 8};
            for (int rr : cand_radix)
                for (int lines : cand_lines)
                    for (int sq = 0; sq < 4; sq++)
                        for (int occ : {0, 4}) {
                        if (!rk4ip::axis_schedule_ok(N, mode, axis, n0, lines, sq, rr, plan->f64, occ ? occ : 1)) continue;
                        Sched cand;
                        cand.lines = lines;
                        cand.seq = sq;
                        cand.radix = rr;
                        cand.occ = occ;
                        float ms = 0.f;
                        int rc = time_pass(plan, g, defs[i], cand, 5, &ms);
                        if (rc) return rc;
                        if (ms < best) {
                            best = ms;
                            pick = cand;
                        }
                    }
            plan->sched[gi][i] = pick;
            fresh.push_back({tune_key(g, i, plan->si), pick});
        }
    }
    if (path && !fresh.empty()) {
        // rewrite the cache: old entries kept verbatim, new ones appended
        std::string body = text;
        size_t close = body.rfind('}');
        if (close == std::string::npos) body = "{\n", close = body.size();
        else body = body.substr(0, close);
        bool has_entry = body.find('[') != std::string::npos;
        for (auto& f : fresh) {
            char line[256];
            std::snprintf(line, sizeof(line), "%s \"%s\": [%d, %d, %d, %d]\n", has_entry ? "," : " ", f.first.c_str(),
                          f.second.lines, f.second.seq, f.second.radix, f.second.occ);
            body += line;
            has_entry = true;
        }
        body += "}\n";
        if (FILE* fh = std::fopen(path, "w")) {
            std::fwrite(body.data(), 1, body.size(), fh);
            std::fclose(fh);
        }
    }
    return RK4IP_OK;
}

// Enqueue `nsteps` steps of every 1D group. step_base != null: step = *step_base + step_off.
// Groups run by the k-space line step keep their state in k-space between launches:
// from_k says it is there at entry (else it is psi), to_k that it stays there at exit (else
// it is transformed back into psi). A zero-step launch only converts. Other 1D groups
// always hold their state in psi.
int enqueue_lines(rk4ip_plan_t plan, hipStream_t stream, float2* psi, int64_t step_off, int64_t nsteps,
                  const int64_t* step_base, bool allow_fuse, bool from_k = false, bool to_k = false) {
    const bool capturing = step_base != nullptr;
    const bool fuse = allow_fuse && (plan->flags & RK4IP_FLAG_FUSE_1D);
    int rc;
    for (size_t gi = 0; gi < plan->groups.size(); gi++) {
        auto& g = plan->groups[gi];
        if (g.p.ndim != 1) continue;
        const int radix = plan->sched[gi][0].radix;
        auto launch = [&](int64_t n, int64_t s0, bool fk, bool tk) {
            const int io = g.kline ? ((fk ? 1 : 0) | (tk ? 2 : 0)) : 0;
            return timed_launch(plan, stream, (int)gi, 0, capturing, [&] {
                return rk4ip::launch_line_step(g.d, psi, (int)n, s0, step_base, plan->f64, radix, plan->si, stream,
                                                io);
            });
        };
        if (nsteps <= 0) {
            if (g.kline && from_k != to_k && (rc = launch(0, step_off, from_k, to_k))) return rc;
            continue;
        }
        if (fuse) {
            if ((rc = launch(nsteps, step_off, from_k, to_k))) return rc;
        } else {
            for (int64_t s = 0; s < nsteps; s++)
                if ((rc = launch(1, step_off + s, s == 0 ? from_k : true, s == nsteps - 1 ? to_k : true))) return rc;
        }
    }
    return RK4IP_OK;
}

// Enqueue part of a run on every 2D/3D group: OPEN at step_off (if `open`), then `nunits`
// units (MID of step s, NEXT into step s + 1, for s = step_off ...), then, if `close`, MID
// and CLOSE of step step_off + nunits. step_base != null: every step index is offset by
// *step_base.
int enqueue_lattice(rk4ip_plan_t plan, hipStream_t stream, float2* psi, int64_t step_off, int64_t nunits, bool open,
                    bool close, const int64_t* step_base) {
    const bool capturing = step_base != nullptr;
    auto launch_role = [&](int role, int64_t step) -> int {
        if (!plan->merged.empty()) {
            // one launch per pass over all groups of a dimensionality (timed under the
            // first group of its work list)
            for (const auto& m : plan->merged) {
                if (m.role != role) continue;
                rk4ip::PassArgs pa{};
                pa.psi = psi;
                pa.twice = m.twice;
                pa.A = plan->A;
                pa.B = plan->B;
                pa.step_off = step;
                pa.step_base = step_base;
                int rc = timed_launch(plan, stream, m.list.gid[0], m.pass, capturing, [&] {
                    return rk4ip::launch_axis_merged(m.list, m.mode, m.axis, m.noise, m.blocks, m.smem, pa, stream);
                });
                if (rc) return rc;
            }
            return RK4IP_OK;
        }
        for (size_t gi = 0; gi < plan->groups.size(); gi++) {
            auto& g = plan->groups[gi];
            if (g.p.ndim == 1) continue;
            PassDef defs[kMaxPasses];
            const int np = pass_list(g.p.ndim, plan->si, defs);
            for (int i = 0; i < np; i++) {
                if (defs[i].role != role) continue;
                rk4ip::PassArgs pa{};
                pa.psi = psi;
                pa.twice = defs[i].twice;
                pa.A = plan->A;
                pa.B = plan->B;
                pa.step_off = step;
                pa.step_base = step_base;
                pa.f64 = plan->f64 ? 1 : 0;
                pa.occ = plan->sched[gi][i].occ;
                pa.lines = plan->sched[gi][i].lines;
                pa.seq = plan->sched[gi][i].seq;
                pa.radix = plan->sched[gi][i].radix;
                int rc = timed_launch(plan, stream, (int)gi, i, capturing, [&] {
                    return rk4ip::launch_axis(g.d, defs[i].axis, defs[i].mode, pa, stream);
                });
                if (rc) return rc;
            }
        }
        return RK4IP_OK;
    };
    int rc;
    if (open && (rc = launch_role(ROLE_OPEN, step_off))) return rc;
    for (int64_t u = 0; u < nunits; u++) {
        if ((rc = launch_role(ROLE_MID, step_off + u))) return rc;
        if ((rc = launch_role(ROLE_NEXT, step_off + u + 1))) return rc;
    }
    if (close) {
        if ((rc = launch_role(ROLE_MID, step_off + nunits))) return rc;
        if ((rc = launch_role(ROLE_CLOSE, step_off + nunits))) return rc;
    }
    return RK4IP_OK;
}

bool has_lattice(rk4ip_plan_t plan) {
    for (auto& g : plan->groups)
        if (g.p.ndim > 1) return true;
    return false;
}

// Enqueue `nsteps` steps (from step index step_off) of every group, eagerly.
int enqueue_steps(rk4ip_plan_t plan, hipStream_t stream, float2* psi, int64_t step_off, int64_t nsteps,
                  bool allow_fuse) {
    if (nsteps <= 0) return RK4IP_OK;
    int rc = enqueue_lines(plan, stream, psi, step_off, nsteps, nullptr, allow_fuse);
    if (rc) return rc;
    if (!has_lattice(plan)) return RK4IP_OK;
    return enqueue_lattice(plan, stream, psi, step_off, nsteps - 1, true, true, nullptr);
}

int device_ok(rk4ip_plan_t plan) {
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count < 1) {
        (void)hipGetLastError();
        return fail(plan, RK4IP_ERR_NO_DEVICE, "no HIP device");
    }
    int dev = 0;
    HIPCHK(plan, hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIPCHK(plan, hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(plan, RK4IP_ERR_NO_DEVICE, std::string("device is ") + prop.gcnArchName + ", not gfx950");
    if (plan) plan->device = dev;
    return RK4IP_OK;
}

// Does the plan hold a cosine / sine group? Only the step (rk4ip_step, rk4ip_run without
// samples) takes those: the other kernels index the lattice as a Fourier line.
bool has_basis_group(rk4ip_plan_t plan) {
    for (auto& g : plan->groups)
        if (g.p.basis) return true;
    return false;
}

int do_diagnostics(rk4ip_plan_t plan, const float2* psi, double* out) {
    if (has_basis_group(plan))
        return fail(plan, RK4IP_ERR_INVALID_ARG, "diagnostics take Fourier groups only");
    for (auto& g : plan->groups) {
        const double* parts[3] = {nullptr, nullptr, nullptr};
        for (int a = 0; a < g.p.ndim; a++) {
            double* part = reinterpret_cast<double*>(plan->ws + g.part_off[a]);
            const double kscale = 2.0 * kPi / (g.p.hi[a] - g.p.lo[a]);
            HIPCHK(plan, rk4ip::launch_diag_axis(g.d, a, psi, kscale, part, plan->stream));
            parts[a] = part;
        }
        rk4ip::DiagConst c{g.dV, g.p.alpha, 0.5 * g.p.g_nl};
        HIPCHK(plan, rk4ip::launch_diag_final(g.d, c, parts[0], parts[1] ? parts[1] : parts[0],
                                              parts[2] ? parts[2] : parts[0], out + g.first_inst * 4, plan->flag,
                                              plan->stream));
    }
    return RK4IP_OK;
}

// Replayed graphs hold 2^level steady-state steps, level < kGraphLevels (at most 32).
constexpr int kGraphLevels = 6;

// Build (or reuse) the graph of gsteps = 2^level steady-state steps whose step index s is
// read from the device counter: the 1D groups' steps s ... s + gsteps - 1 and the 2D/3D
// groups' units (MID of step s + u, NEXT into s + u + 1), followed by counter += gsteps.
// A run of any length replays the binary decomposition of its units, so runs of
// different lengths share the recorded graphs.
int ensure_graph(rk4ip_plan_t plan, float2* psi, int level) {
    if (plan->graph_psi != psi) drop_step_graphs(plan);
    if (plan->graph[level]) return RK4IP_OK;
    const int gsteps = 1 << level;
    // record on a private stream (the caller's may be the legacy default stream, which
    // cannot be captured); the instantiated graph is then launched on the plan's stream
    if (!plan->capture_stream) HIPCHK(plan, hipStreamCreateWithFlags(&plan->capture_stream, hipStreamNonBlocking));
    hipStream_t s = plan->capture_stream;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return fail_hip(plan, e, "hipStreamBeginCapture");
    int rc = enqueue_lines(plan, s, psi, 0, gsteps, plan->counter, true, true, true);
    if (rc == RK4IP_OK) rc = enqueue_lattice(plan, s, psi, 0, gsteps, false, false, plan->counter);
    hipError_t e2 = rk4ip::launch_counter(plan->counter, gsteps, 1, s);
    hipGraph_t gr = nullptr;
    hipError_t e3 = hipStreamEndCapture(s, &gr);
    if (rc != RK4IP_OK || e2 != hipSuccess || e3 != hipSuccess || !gr) {
        if (gr) (void)hipGraphDestroy(gr);
        plan->err = "graph capture failed";
        return RK4IP_ERR_NOT_CAPTURABLE;
    }
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(gr);
        plan->err = std::string("hipGraphInstantiate: ") + hipGetErrorString(e);
        return RK4IP_ERR_NOT_CAPTURABLE;
    }
    plan->graph[level] = ex;
    plan->graph_src[level] = gr;
    plan->graph_psi = psi;
    // upload it now (on the plan's stream, ahead of the run's work) rather than at its first
    // launch, which may fall inside a timed run
    e = hipGraphUpload(ex, plan->stream);
    if (e != hipSuccess) return fail_hip(plan, e, "hipGraphUpload");
    return RK4IP_OK;
}

// Advance nsteps from step index `step`, replaying graphs of steady-state steps when
// enabled: OPEN, graphs, the remaining units eagerly, CLOSE.
int advance(rk4ip_plan_t plan, float2* psi, int64_t step, int64_t nsteps) {
    if (nsteps <= 0) return RK4IP_OK;
    if (!(plan->flags & RK4IP_FLAG_GRAPH)) return enqueue_steps(plan, plan->stream, psi, step, nsteps, true);
    const bool lattice = has_lattice(plan);
    const int64_t units = lattice ? nsteps - 1 : nsteps;
    int rc;
    if (lattice && (rc = enqueue_lattice(plan, plan->stream, psi, step, 0, true, false, nullptr))) return rc;
    int64_t done = 0;
    if (units >= 1) {
        // every level is recorded on the first replayed run of a field, before that run's
        // first replay, so that a later run of another length records nothing
        if (plan->graph_psi != psi)
            for (int level = 0; level < kGraphLevels; level++)
                if ((rc = ensure_graph(plan, psi, level))) return rc;
        HIPCHK(plan, rk4ip::launch_counter(plan->counter, step, 0, plan->stream));
        // the replays step the k-space lines' states in the workspace
        if ((rc = enqueue_lines(plan, plan->stream, psi, step, 0, nullptr, true, false, true))) return rc;
        while (done < units) {
            int level = kGraphLevels - 1;
            while ((int64_t(1) << level) > units - done) level--;
            if ((rc = ensure_graph(plan, psi, level))) return rc;
            hipError_t e = hipGraphLaunch(plan->graph[level], plan->stream);
            if (e != hipSuccess) {
                plan->err = std::string("hipGraphLaunch: ") + hipGetErrorString(e);
                return RK4IP_ERR_NOT_CAPTURABLE;
            }
            done += int64_t(1) << level;
        }
    }
    if ((rc = enqueue_lines(plan, plan->stream, psi, step + done, nsteps - done, nullptr, true, done > 0, false)))
        return rc;
    if (lattice) return enqueue_lattice(plan, plan->stream, psi, step + done, units - done, false, true, nullptr);
    return RK4IP_OK;
}

// ---------------------------------------------------------------- the no-allocation step
//
// rk4ip_step_noalloc keeps its tables and work fields in `scratch`, a file-scope device
// array that every GPU the library runs on holds for the life of the process. In host code
// the array's name is not a device address: its address is taken once per device with
// hipGetSymbolAddress (with that device current) and only that pointer is used.
constexpr size_t kNoallocBytes = RK4IP_NOALLOC_SCRATCH_BYTES;
constexpr int kNoallocMaxGroups = 16;
constexpr int kNoallocMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

struct NoallocDevice {
    std::once_flag once;
    char* ptr = nullptr;
    int status = RK4IP_ERR_NO_DEVICE;
};
NoallocDevice g_noalloc[kNoallocMaxDevices];

// The scratch address of the current device (and whether it is a gfx950), looked up once.
int noalloc_scratch(char** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNoallocMaxDevices) {
        (void)hipGetLastError();
        return RK4IP_ERR_NO_DEVICE;
    }
    NoallocDevice& nd = g_noalloc[dev];
    std::call_once(nd.once, [&] {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess || std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
            (void)hipGetLastError();
            nd.status = RK4IP_ERR_NO_DEVICE;
            return;
        }
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            nd.status = RK4IP_ERR_HIP;
            return;
        }
        nd.ptr = static_cast<char*>(ptr);
        nd.status = RK4IP_OK;
    });
    *out = nd.ptr;
    return nd.status;
}

// The tables of build_basis_tables computed on the device in FP64 (the same expressions, in
// the same order, without contraction), one thread per entry m; kpl = pi / L.
__global__ void k_noalloc_basis_tables(double2* __restrict__ T1, float2* __restrict__ tw, double2* __restrict__ T2, int n,
                                       double kpl, double alpha, double h, double gamma, int basis) {
#pragma clang fp contract(off)
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    const double damp = exp(-gamma * h / 2.0), em1 = expm1(-gamma * h / 2.0);
    const double inv_n = 1.0 / (double)n;
    auto em1_of = [&](int mm, double& c, double& s) {
        const double k = kpl * (double)(basis == 1 ? mm : n - mm);
        const double theta = alpha * k * k * h / 2.0;
        const double sh = sin(theta / 2.0);
        c = em1 - 2.0 * damp * sh * sh;
        s = -damp * sin(theta);
    };
    double ac, as;
    em1_of(m, ac, as);
    if (m == 0) {
        T1[m] = make_double2(ac * inv_n, as * inv_n);
        T2[m] = make_double2(0.0, 0.0);
    } else {
        double bc, bs;
        em1_of(n - m, bc, bs);
        const double dc = 0.5 * (ac - bc), ds = 0.5 * (as - bs);
        const double ph = kPi * (double)m / (double)n;
        const double cp = cos(ph), sp = sin(ph);
        T1[m] = make_double2(0.5 * (ac + bc) * inv_n, 0.5 * (as + bs) * inv_n);
        T2[m] = make_double2((dc * cp - ds * sp) * inv_n, (dc * sp + ds * cp) * inv_n);
    }
    const double ang = 2.0 * kPi * (double)m / (double)n;
    tw[m] = make_float2((float)cos(ang), (float)-sin(ang));
}

// The tables of build_tables computed on the device in FP64 (the same expressions, in the
// same order, without contraction), one thread per entry m: (E - 1)/n, the twiddles and,
// when E2 is not null, (e^{L h} - 1)/n. kscale = 2 pi / L; gamma is the damping of this axis
// (zero off axis 0).
__global__ void k_noalloc_tables(float2* __restrict__ E, float2* __restrict__ tw, float2* __restrict__ E2, int n,
                                 double kscale, double alpha, double h, double gamma) {
#pragma clang fp contract(off)
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    const double damp = exp(-gamma * h / 2.0);
    const double em1 = expm1(-gamma * h / 2.0);
    const double inv_n = 1.0 / (double)n;
    const double k = kscale * (double)(m < n / 2 ? m : m - n);
    const double theta = alpha * k * k * h / 2.0;
    const double sh = sin(theta / 2.0);
    const double c = em1 - 2.0 * damp * sh * sh;
    const double sn = -damp * sin(theta);
    E[m] = make_float2((float)(c * inv_n), (float)(sn * inv_n));
    const double ang = 2.0 * kPi * (double)m / (double)n;
    tw[m] = make_float2((float)cos(ang), (float)-sin(ang));
    if (E2) {
        const double d2 = damp * damp, em2 = expm1(-gamma * h), st = sin(theta);
        const double c2 = em2 - 2.0 * d2 * st * st;
        const double s2 = -d2 * sin(2.0 * theta);
        E2[m] = make_float2((float)(c2 * inv_n), (float)(s2 * inv_n));
    }
}

// One step of every group from src into dst (the adjoint's recompute: the states of a
// segment go straight into their slots). Per-group launches with the plan's schedules;
// step_base != null: the step index is *step_base + step_off.
int enqueue_step_to(rk4ip_plan_t plan, hipStream_t st, const float2* src, float2* dst, int64_t step_off,
                    const int64_t* step_base) {
    for (size_t gi = 0; gi < plan->groups.size(); gi++) {
        auto& g = plan->groups[gi];
        if (g.p.ndim == 1) {
            HIPCHK(plan, rk4ip::launch_line_step(g.d, const_cast<float2*>(src), 1, step_off, step_base, plan->f64,
                                                 plan->sched[gi][0].radix, plan->si, st, 0, dst));
            continue;
        }
        PassDef defs[kMaxPasses];
        const int np = pass_list(g.p.ndim, plan->si, defs);
        for (int role : {ROLE_OPEN, ROLE_MID, ROLE_CLOSE}) {
            for (int i = 0; i < np; i++) {
                if (defs[i].role != role) continue;
                rk4ip::PassArgs pa{};
                pa.psi = const_cast<float2*>(src);
                pa.psi_out = dst;
                pa.A = plan->A;
                pa.B = plan->B;
                pa.step_off = step_off;
                pa.step_base = step_base;
                pa.twice = defs[i].twice;
                pa.f64 = plan->f64 ? 1 : 0;
                pa.occ = plan->sched[gi][i].occ;
                pa.lines = plan->sched[gi][i].lines;
                pa.seq = plan->sched[gi][i].seq;
                pa.radix = plan->sched[gi][i].radix;
                HIPCHK(plan, rk4ip::launch_axis(g.d, defs[i].axis, defs[i].mode, pa, st));
            }
        }
    }
    return RK4IP_OK;
}

// The adjoint of one step at state pn (psi_n) for every group: lam <- (d step)^T lam, and
// the potential gradient accumulated into vbar. W, X, Y: work fields.
int enqueue_adjoint_step(rk4ip_plan_t plan, hipStream_t st, const float2* pn, float2* lam, double* vbar, float2* W,
                         float2* X, float2* Y, int64_t step_off, const int64_t* step_base) {
    for (auto& g : plan->groups) {
        if (g.p.ndim == 1) {
            HIPCHK(plan, rk4ip::launch_line_adjoint(g.d, pn, lam, vbar, step_off, step_base, st));
            continue;
        }
        const int last = g.p.ndim - 1;
        rk4ip::PassArgs pa{};
        pa.step_off = step_off;
        pa.step_base = step_base;
        // forward: (A, B) = D (psi_n, hG(psi_n)) = (a, k1); the last axis's pass also forms
        // u = a + k3 and W = D_last u
        pa.psi = const_cast<float2*>(pn);
        pa.A = plan->A;
        pa.B = plan->B;
        HIPCHK(plan, rk4ip::launch_axis(g.d, 0, rk4ip::PASS_FIRST, pa, st));
        for (int a = 1; a < last; a++) HIPCHK(plan, rk4ip::launch_axis(g.d, a, rk4ip::PASS_D2, pa, st));
        rk4ip::PassArgs pd = pa;
        pd.psi = W;
        HIPCHK(plan, rk4ip::launch_axis_adjoint(g.d, last, rk4ip::PASS_D2U, pd, st));
        // forward: W = D (a + k3) on the middle axes; axis 0 is applied in the next pass
        rk4ip::PassArgs pu{};
        pu.step_off = step_off;
        pu.step_base = step_base;
        pu.psi = W;
        for (int a = last - 1; a >= 1; a--) HIPCHK(plan, rk4ip::launch_axis(g.d, a, rk4ip::PASS_D1, pu, st));
        // adjoint: w = D_0 W, (X, Y) = D^T (lam, h J(w)^T lam/6), then the stage transposes
        rk4ip::PassArgs pw{};
        pw.step_off = step_off;
        pw.step_base = step_base;
        pw.adj = 1;
        pw.psi = lam;
        pw.aux0 = W;
        pw.A = X;
        pw.B = Y;
        pw.vbar = vbar;
        HIPCHK(plan, rk4ip::launch_axis_adjoint(g.d, 0, rk4ip::PASS_XAW, pw, st));
        for (int a = 1; a < last; a++) HIPCHK(plan, rk4ip::launch_axis(g.d, a, rk4ip::PASS_D2, pw, st));
        pw.aux0 = plan->A;
        pw.aux1 = plan->B;
        HIPCHK(plan, rk4ip::launch_axis(g.d, last, rk4ip::PASS_AS, pw, st));
        // adjoint: lam = D^T abar + h J(psi_n)^T D^T k1bar (AS applied the last axis's
        // share, AF applies axis 0's)
        rk4ip::PassArgs pf{};
        pf.step_off = step_off;
        pf.step_base = step_base;
        pf.adj = 1;
        pf.A = X;
        pf.B = Y;
        pf.psi = lam;
        pf.aux0 = pn;
        pf.vbar = vbar;
        for (int a = 1; a < last; a++) HIPCHK(plan, rk4ip::launch_axis(g.d, a, rk4ip::PASS_D2, pf, st));
        HIPCHK(plan, rk4ip::launch_axis(g.d, 0, rk4ip::PASS_AF, pf, st));
    }
    return RK4IP_OK;
}

// Record `body` (enqueueing on the given stream) as a graph on the plan's private stream.
template <class Fn>
int record_graph(rk4ip_plan_t plan, hipGraphExec_t* out, Fn&& body) {
    if (!plan->capture_stream) HIPCHK(plan, hipStreamCreateWithFlags(&plan->capture_stream, hipStreamNonBlocking));
    hipStream_t s = plan->capture_stream;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return fail_hip(plan, e, "hipStreamBeginCapture");
    const int rc = body(s);
    hipGraph_t gr = nullptr;
    const hipError_t e2 = hipStreamEndCapture(s, &gr);
    if (rc != RK4IP_OK || e2 != hipSuccess || !gr) {
        if (gr) (void)hipGraphDestroy(gr);
        plan->err = "graph capture failed";
        return RK4IP_ERR_NOT_CAPTURABLE;
    }
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (e != hipSuccess) {
        plan->err = std::string("hipGraphInstantiate: ") + hipGetErrorString(e);
        return RK4IP_ERR_NOT_CAPTURABLE;
    }
    *out = ex;
    return RK4IP_OK;
}

}  // namespace

// ================================================================== C ABI

extern "C" {

const char* rk4ip_strerror(int status) {
    switch (status) {
        case RK4IP_OK: return "ok";
        case RK4IP_ERR_INVALID_ARG: return "invalid argument";
        case RK4IP_ERR_UNSUPPORTED_SHAPE: return "unsupported lattice shape";
        case RK4IP_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
        case RK4IP_ERR_HIP: return "HIP runtime error";
        case RK4IP_ERR_NONFINITE: return "non-finite value in a field";
        case RK4IP_ERR_NOT_CAPTURABLE: return "graph capture or replay failed";
        case RK4IP_ERR_NO_DEVICE: return "no usable gfx950 device";
        default: return "unknown status";
    }
}

size_t rk4ip_workspace_bytes(const rk4ip_problem* probs, int nprob, uint32_t flags) {
    if (validate(probs, nprob, flags) != RK4IP_OK) return 0;
    return layout(probs, nprob, flags, nullptr).total;
}

int rk4ip_plan(const rk4ip_problem* probs, int nprob, void* workspace, size_t ws_bytes, void* stream,
               uint32_t flags, rk4ip_plan_t* out) {
    if (!out) return RK4IP_ERR_INVALID_ARG;
    *out = nullptr;
    int rc = validate(probs, nprob, flags);
    if (rc != RK4IP_OK) return rc;
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0) return RK4IP_ERR_INVALID_ARG;
    std::vector<GroupHost> gh(nprob);
    Layout L = layout(probs, nprob, flags, gh.data());
    if (ws_bytes < L.total) return RK4IP_ERR_WORKSPACE_TOO_SMALL;

    rk4ip_plan_s* plan = new (std::nothrow) rk4ip_plan_s();
    if (!plan) return RK4IP_ERR_INVALID_ARG;
    rc = device_ok(plan);
    if (rc != RK4IP_OK) {
        delete plan;
        return rc;
    }
    plan->ws = static_cast<char*>(workspace);
    plan->ws_bytes = ws_bytes;
    plan->stream = static_cast<hipStream_t>(stream);
    plan->flags = flags;
    plan->f64 = (flags & RK4IP_FLAG_FP64_TRANSFORMS) != 0;
    plan->si = (flags & RK4IP_FLAG_SEMI_IMPLICIT) != 0;
    plan->points = L.points;
    plan->counter = reinterpret_cast<int64_t*>(plan->ws + L.header);
    plan->flag = reinterpret_cast<int*>(plan->ws + L.header + 64);
    plan->A = reinterpret_cast<float2*>(plan->ws + L.fields);
    plan->B = plan->A + L.points;

    // host staging of the tables; uploaded with one synchronous copy per table
    int64_t offset = 0, inst = 0;
    for (int i = 0; i < nprob; i++) {
        GroupHost& g = gh[i];
        g.p = probs[i];
        const rk4ip_problem& p = g.p;
        GroupDev& d = g.d;
        fill_group(g, plan->ws, flags, offset);
        for (int a = 0; a < p.ndim; a++) {
            std::vector<float2> E, tw, E2;
            std::vector<double2> E64, tw64;
            const bool kline = g.kline;
            std::vector<double2> T12;
            if (g.dct) {
                build_basis_tables(p, T12, tw);
                E.assign(tw.size(), make_float2(0.f, 0.f));  // unused by the cosine / sine line
            } else {
                build_tables(transform_problem(p, flags), a, E, tw, plan->f64 ? &E64 : nullptr,
                             plan->f64 ? &tw64 : nullptr, kline ? &E2 : nullptr);
            }
            hipError_t e1 = hipMemcpy(plan->ws + g.tab_off[a], E.data(), sizeof(float2) * E.size(), hipMemcpyHostToDevice);
            hipError_t e2 = hipMemcpy(plan->ws + g.tw_off[a], tw.data(), sizeof(float2) * tw.size(), hipMemcpyHostToDevice);
            if (e1 == hipSuccess && e2 == hipSuccess && kline)
                e1 = hipMemcpy(plan->ws + g.e2_off, E2.data(), sizeof(float2) * E2.size(), hipMemcpyHostToDevice);
            if (e1 == hipSuccess && e2 == hipSuccess && g.dct)
                e1 = hipMemcpy(plan->ws + g.e2_off, T12.data(), sizeof(double2) * T12.size(), hipMemcpyHostToDevice);
            if (e1 == hipSuccess && e2 == hipSuccess && plan->f64) {
                e1 = hipMemcpy(plan->ws + g.tab64_off[a], E64.data(), sizeof(double2) * E64.size(),
                               hipMemcpyHostToDevice);
                e2 = hipMemcpy(plan->ws + g.tw64_off[a], tw64.data(), sizeof(double2) * tw64.size(),
                               hipMemcpyHostToDevice);
            }
            if (e1 != hipSuccess || e2 != hipSuccess) {
                rc = fail_hip(plan, e1 != hipSuccess ? e1 : e2, "table upload");
                release_plan(plan);
                return rc;
            }
        }
        if (p.conv_K) {
            std::vector<float2> kh;
            build_conv_table(p, g.dV, kh);
            hipError_t e1 = hipMemcpy(plan->ws + g.conv_off, kh.data(), sizeof(float2) * kh.size(),
                                      hipMemcpyHostToDevice);
            if (e1 != hipSuccess) {
                rc = fail_hip(plan, e1, "table upload");
                release_plan(plan);
                return rc;
            }
        }
        (void)d;
        g.first_inst = inst;
        offset += p.batch * g.M;
        inst += p.batch;
        {
            PassDef defs[kMaxPasses];
            plan->sched.push_back(std::vector<Sched>(p.ndim == 1 ? 1 : pass_list(p.ndim, plan->si, defs)));
        }
    }
    plan->ninst = inst;
    plan->groups = std::move(gh);
    if (flags & RK4IP_FLAG_MERGE_GROUPS) {
        rc = build_merged(plan, L.gdev);
        if (rc != RK4IP_OK) {
            release_plan(plan);
            return rc;
        }
    }
    if (plan->f64) {
        // FP64 transforms have no implicit default tile: take the first compiled candidate
        for (size_t gi = 0; gi < plan->groups.size(); gi++) {
            const GroupHost& g = plan->groups[gi];
            if (g.p.ndim == 1) continue;
            PassDef defs[kMaxPasses];
            const int np = pass_list(g.p.ndim, plan->si, defs);
            for (int k = 0; k < np; k++) {
                if (!default_f64_sched(g, defs[k].axis, defs[k].mode, &plan->sched[gi][k])) {
                    release_plan(plan);
                    return RK4IP_ERR_UNSUPPORTED_SHAPE;
                }
            }
        }
    }
    if (flags & RK4IP_FLAG_AUTOTUNE) {
        rc = autotune(plan);
        if (rc != RK4IP_OK) {
            release_plan(plan);
            return rc;
        }
    }
    // names of the chosen schedules
    for (size_t gi = 0; gi < plan->groups.size(); gi++) {
        const rk4ip_problem& p = plan->groups[gi].p;
        char name[160];
        std::vector<std::string> names;
        if (p.ndim == 1) {
            const int rr = plan->f64 ? 8 : (plan->sched[gi][0].radix ? plan->sched[gi][0].radix : 16);
            std::snprintf(name, sizeof(name), "%s:n%lld:r%d%s", plan->si ? "line_si" : "line_step", (long long)p.n[0], rr,
                          plan->f64 ? ":f64" : "");
            names.push_back(name);
        } else {
            PassDef defs[kMaxPasses];
            const int np = pass_list(p.ndim, plan->si, defs);
            for (int k = 0; k < np; k++) {
                const int a = defs[k].axis;
                const Sched sc = plan->sched[gi][k];
                const int lines = sc.lines ? sc.lines : rk4ip::axis_lines((int)p.n[a], a, (int)p.n[0]);
                std::snprintf(name, sizeof(name), "%s%s:axis%d:n%lld:%s:lines%d:%s:r%d%s%s", mode_name(defs[k].mode),
                              defs[k].twice ? "x2" : "", a, (long long)p.n[a], a == 0 ? "contig" : "strided", lines,
                              sc.seq == 3 ? "split" : (sc.seq == 2 ? "seq-deferred" : (sc.seq ? "seq" : "joint")), sc.radix ? sc.radix : 16,
                              sc.occ == 4 ? ":o4" : "", plan->f64 ? ":f64" : "");
                names.push_back(name);
            }
        }
        plan->sched_names.push_back(names);
    }
    hipError_t e = hipMemset(plan->ws + L.header, 0, kAlign);
    if (e != hipSuccess) {
        rc = fail_hip(plan, e, "hipMemset");
        release_plan(plan);
        return rc;
    }
    *out = plan;
    return RK4IP_OK;
}

int rk4ip_set_stream(rk4ip_plan_t plan, void* stream) {
    if (!plan) return RK4IP_ERR_INVALID_ARG;
    if (plan->stream != static_cast<hipStream_t>(stream)) drop_graph(plan);
    plan->stream = static_cast<hipStream_t>(stream);
    return RK4IP_OK;
}

int rk4ip_step(rk4ip_plan_t plan, void* psi, int64_t step_index) {
    if (!plan || !psi || step_index < 0) return RK4IP_ERR_INVALID_ARG;
    return enqueue_steps(plan, plan->stream, static_cast<float2*>(psi), step_index, 1, false);
}

int rk4ip_diagnostics(rk4ip_plan_t plan, const void* psi, double* out) {
    if (!plan || !psi || !out) return RK4IP_ERR_INVALID_ARG;
    return do_diagnostics(plan, static_cast<const float2*>(psi), out);
}

int rk4ip_run(rk4ip_plan_t plan, void* psi_v, int64_t step0, int64_t nsteps, int64_t sample_every, double* diag,
              void* ckpt_v, int64_t ckpt_every) {
    if (!plan || !psi_v || step0 < 0 || nsteps < 0) return RK4IP_ERR_INVALID_ARG;
    if (diag && sample_every < 1) return RK4IP_ERR_INVALID_ARG;
    if (ckpt_v && ckpt_every < 1) return RK4IP_ERR_INVALID_ARG;
    float2* psi = static_cast<float2*>(psi_v);
    float2* ckpt = static_cast<float2*>(ckpt_v);
    const int64_t se = diag ? sample_every : 0;
    const int64_t ce = ckpt ? ckpt_every : 0;
    int64_t s = 0;
    int64_t sample = 0;
    while (true) {
        if (se && s % se == 0) {
            int rc = do_diagnostics(plan, psi, diag + sample * plan->ninst * 4);
            if (rc) return rc;
            sample++;
        }
        if (s == nsteps) break;
        if (ce && s % ce == 0)
            HIPCHK(plan, hipMemcpyAsync(ckpt + (s / ce) * plan->points, psi, sizeof(float2) * plan->points,
                                        hipMemcpyDeviceToDevice, plan->stream));
        // run to the next sample or checkpoint boundary
        int64_t next = nsteps;
        if (se) next = std::min(next, (s / se + 1) * se);
        if (ce) next = std::min(next, (s / ce + 1) * ce);
        int rc = advance(plan, psi, step0 + s, next - s);
        if (rc) return rc;
        s = next;
    }
    return RK4IP_OK;
}

int rk4ip_overlap(rk4ip_plan_t plan, int group, const void* phi, const void* psi, double* out) {
    if (!plan || !phi || !psi || !out || group < 0 || group >= (int)plan->groups.size()) return RK4IP_ERR_INVALID_ARG;
    if (plan->groups[group].p.basis) return fail(plan, RK4IP_ERR_INVALID_ARG, "overlaps take Fourier groups only");
    const GroupHost& g = plan->groups[group];
    HIPCHK(plan, rk4ip::launch_overlap(g.d, g.dV, static_cast<const float2*>(phi), static_cast<const float2*>(psi), out,
                                       plan->stream));
    return RK4IP_OK;
}

int rk4ip_moments(rk4ip_plan_t plan, int group, const void* psi, double* mean, double* var) {
    if (!plan || !psi || !mean || !var || group < 0 || group >= (int)plan->groups.size()) return RK4IP_ERR_INVALID_ARG;
    if (plan->groups[group].p.basis) return fail(plan, RK4IP_ERR_INVALID_ARG, "moments take Fourier groups only");
    const GroupHost& g = plan->groups[group];
    HIPCHK(plan, rk4ip::launch_moments(g.d, static_cast<const float2*>(psi), mean, var, plan->stream));
    return RK4IP_OK;
}

int rk4ip_ark45(rk4ip_plan_t plan, void* psi_v, double t_span, double tol, int64_t max_attempts, double* h,
                int64_t* stats, double* h_log, int64_t log_cap, int explicit_L) {
    if (!plan || !psi_v || !h || !stats || !(t_span >= 0.0) || !std::isfinite(t_span) || !(tol > 0.0) ||
        !std::isfinite(tol) || max_attempts < 1 || log_cap < 0 || (log_cap > 0) != (h_log != nullptr))
        return RK4IP_ERR_INVALID_ARG;
    for (auto& g : plan->groups) {
        if (g.p.ndim != 1) return fail(plan, RK4IP_ERR_UNSUPPORTED_SHAPE, "the adaptive integrator takes 1D groups");
        if (g.p.sigma != 0.0 || g.p.sigma_V != 0.0)
            return fail(plan, RK4IP_ERR_INVALID_ARG, "the adaptive integrator is deterministic");
        if (g.p.basis) return fail(plan, RK4IP_ERR_INVALID_ARG, "the adaptive integrator takes Fourier groups");
    }
    float2* psi = static_cast<float2*>(psi_v);
    for (auto& g : plan->groups) {
        rk4ip::ArkArgs x{};
        x.t_span = t_span;
        x.tol = tol;
        x.alpha = g.p.alpha;
        x.gamma = g.p.gamma;
        x.kscale = 2.0 * kPi / (g.p.hi[0] - g.p.lo[0]);
        x.max_attempts = max_attempts;
        x.inst_base = g.first_inst;
        x.log_cap = log_cap;
        x.h = h;
        x.stats = stats;
        x.h_log = h_log;
        x.explicit_L = explicit_L ? 1 : 0;
        HIPCHK(plan, rk4ip::launch_line_ark45(g.d, psi, x, plan->stream));
    }
    return RK4IP_OK;
}

size_t rk4ip_adjoint_workspace_bytes(rk4ip_plan_t plan, int64_t ckpt_every) {
    if (!plan || ckpt_every < 1) return 0;
    // segment states, the adjoint state, three work fields (w, and the adjoint pair) and
    // the FP64 potential-gradient accumulator
    const size_t field = align_up(sizeof(float2) * (size_t)plan->points);
    return (size_t)(ckpt_every + 4) * field + align_up(sizeof(double) * (size_t)plan->points);
}

int rk4ip_adjoint(rk4ip_plan_t plan, const void* ckpt_v, int64_t step0, int64_t nsteps, int64_t ckpt_every,
                  const void* lambda_T, void* grad_psi0, float* grad_V, void* adj_ws, size_t adj_ws_bytes) {
    if (!plan || !ckpt_v || !lambda_T || !grad_psi0 || !adj_ws || step0 < 0 || nsteps < 0 || ckpt_every < 1)
        return RK4IP_ERR_INVALID_ARG;
    if ((reinterpret_cast<uintptr_t>(adj_ws) % kAlign) != 0) return RK4IP_ERR_INVALID_ARG;
    if (plan->si) return fail(plan, RK4IP_ERR_INVALID_ARG, "the adjoint covers the RK4 step only");
    if (has_basis_group(plan)) return fail(plan, RK4IP_ERR_INVALID_ARG, "the adjoint takes Fourier groups only");
    for (auto& g : plan->groups)
        if (g.p.sigma_V != 0.0 || g.p.conv_K)
            return fail(plan, RK4IP_ERR_INVALID_ARG, "the adjoint covers the local, noise-free potential only");
    if (adj_ws_bytes < rk4ip_adjoint_workspace_bytes(plan, ckpt_every)) return RK4IP_ERR_WORKSPACE_TOO_SMALL;
    hipStream_t st = plan->stream;
    const size_t field = align_up(sizeof(float2) * (size_t)plan->points);
    const int64_t fstride = (int64_t)(field / sizeof(float2));
    char* w = static_cast<char*>(adj_ws);
    float2* store = reinterpret_cast<float2*>(w);  // the states of a segment, slot i = step i
    float2* W = reinterpret_cast<float2*>(w + (size_t)ckpt_every * field);
    float2* X = reinterpret_cast<float2*>(w + (size_t)(ckpt_every + 1) * field);
    float2* Y = reinterpret_cast<float2*>(w + (size_t)(ckpt_every + 2) * field);
    float2* lam = reinterpret_cast<float2*>(w + (size_t)(ckpt_every + 3) * field);  // the adjoint state
    double* vbar = reinterpret_cast<double*>(w + (size_t)(ckpt_every + 4) * field);
    const float2* ckpt = static_cast<const float2*>(ckpt_v);
    const size_t fbytes = sizeof(float2) * (size_t)plan->points;
    HIPCHK(plan, hipMemcpyAsync(lam, lambda_T, fbytes, hipMemcpyDeviceToDevice, st));
    HIPCHK(plan, hipMemsetAsync(vbar, 0, sizeof(double) * (size_t)plan->points, st));

    // With RK4IP_FLAG_GRAPH a whole segment (ckpt_every steps) is two graph replays: the
    // recompute from slot 0 and the backward walk, with step indices read from the device
    // counter. Recorded once per workspace (every buffer they touch lives in it).
    const int64_t M = ckpt_every;
    const bool graphs = (plan->flags & RK4IP_FLAG_GRAPH) != 0 && nsteps >= M;
    if (graphs && (plan->adj_M != M || plan->adj_key[0] != store || plan->adj_key[1] != lam || plan->adj_key[2] != vbar)) {
        if (plan->adj_fwd) (void)hipGraphExecDestroy(plan->adj_fwd);
        if (plan->adj_bwd) (void)hipGraphExecDestroy(plan->adj_bwd);
        plan->adj_fwd = plan->adj_bwd = nullptr;
        plan->adj_M = 0;
        int rc = RK4IP_OK;
        if (M > 1)
            rc = record_graph(plan, &plan->adj_fwd, [&](hipStream_t s) {
                for (int64_t i = 0; i + 1 < M; i++) {
                    const int r = enqueue_step_to(plan, s, store + i * fstride, store + (i + 1) * fstride, i, plan->counter);
                    if (r) return r;
                }
                return (int)RK4IP_OK;
            });
        if (rc == RK4IP_OK)
            rc = record_graph(plan, &plan->adj_bwd, [&](hipStream_t s) {
                for (int64_t i = M - 1; i >= 0; i--) {
                    const int r = enqueue_adjoint_step(plan, s, store + i * fstride, lam, vbar, W, X, Y, i, plan->counter);
                    if (r) return r;
                }
                return (int)RK4IP_OK;
            });
        if (rc != RK4IP_OK) return rc;
        plan->adj_M = M;
        plan->adj_key[0] = store;
        plan->adj_key[1] = lam;
        plan->adj_key[2] = vbar;
    }

    const int64_t nseg = (nsteps + M - 1) / M;
    for (int64_t seg = nseg - 1; seg >= 0; seg--) {
        const int64_t s0 = seg * M;
        const int64_t len = std::min(M, nsteps - s0);
        HIPCHK(plan, hipMemcpyAsync(store, ckpt + seg * plan->points, fbytes, hipMemcpyDeviceToDevice, st));
        if (graphs && len == M) {
            HIPCHK(plan, rk4ip::launch_counter(plan->counter, step0 + s0, 0, st));
            if (plan->adj_fwd) HIPCHK(plan, hipGraphLaunch(plan->adj_fwd, st));
            HIPCHK(plan, hipGraphLaunch(plan->adj_bwd, st));
            continue;
        }
        // recompute the segment's states into their slots, then walk it backwards
        int rc;
        for (int64_t i = 0; i + 1 < len; i++)
            if ((rc = enqueue_step_to(plan, st, store + i * fstride, store + (i + 1) * fstride, step0 + s0 + i, nullptr)))
                return rc;
        for (int64_t i = len - 1; i >= 0; i--)
            if ((rc = enqueue_adjoint_step(plan, st, store + i * fstride, lam, vbar, W, X, Y, step0 + s0 + i, nullptr)))
                return rc;
    }
    HIPCHK(plan, hipMemcpyAsync(grad_psi0, lam, fbytes, hipMemcpyDeviceToDevice, st));
    if (grad_V) HIPCHK(plan, rk4ip::launch_vbar_to_float(vbar, grad_V, plan->points, st));
    return RK4IP_OK;
}

int rk4ip_status(rk4ip_plan_t plan) {
    if (!plan) return RK4IP_ERR_INVALID_ARG;
    hipError_t e = hipStreamSynchronize(plan->stream);
    if (e != hipSuccess) return fail_hip(plan, e, "hipStreamSynchronize");
    int flag = 0;
    e = hipMemcpy(&flag, plan->flag, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail_hip(plan, e, "hipMemcpy(flag)");
    int rc = plan->sticky;
    if (rc == RK4IP_OK && flag) rc = RK4IP_ERR_NONFINITE;
    if (flag) {
        e = hipMemset(plan->flag, 0, sizeof(int));
        if (e != hipSuccess) return fail_hip(plan, e, "hipMemset(flag)");
    }
    plan->sticky = RK4IP_OK;
    return rc;
}

int rk4ip_destroy(rk4ip_plan_t plan) {
    if (!plan) return RK4IP_ERR_INVALID_ARG;
    release_plan(plan);
    return RK4IP_OK;
}

const char* rk4ip_last_error(rk4ip_plan_t plan) { return plan ? plan->err.c_str() : ""; }

int rk4ip_num_passes(rk4ip_plan_t plan, int group) {
    if (!plan || group < 0 || group >= (int)plan->groups.size()) return RK4IP_ERR_INVALID_ARG;
    return (int)plan->sched_names[group].size();
}

const char* rk4ip_schedule(rk4ip_plan_t plan, int group, int pass) {
    if (!plan || group < 0 || group >= (int)plan->groups.size()) return nullptr;
    if (pass < 0 || pass >= (int)plan->sched_names[group].size()) return nullptr;
    return plan->sched_names[group][pass].c_str();
}

int rk4ip_profile(rk4ip_plan_t plan, int enable) {
    if (!plan) return RK4IP_ERR_INVALID_ARG;
    int rc = collect_profile(plan);
    if (rc) return rc;
    plan->profiling = enable != 0;
    plan->prof_ms.assign(plan->groups.size(), std::vector<double>(6, 0.0));
    plan->prof_n.assign(plan->groups.size(), std::vector<int64_t>(6, 0));
    return RK4IP_OK;
}

int rk4ip_profile_read(rk4ip_plan_t plan, int group, int pass, int64_t* count, double* mean_ms) {
    if (!plan || !count || !mean_ms || group < 0 || group >= (int)plan->groups.size()) return RK4IP_ERR_INVALID_ARG;
    if (pass < 0 || pass >= (int)plan->sched_names[group].size()) return RK4IP_ERR_INVALID_ARG;
    int rc = collect_profile(plan);
    if (rc) return rc;
    if (plan->prof_n.empty()) {
        *count = 0;
        *mean_ms = 0.0;
        return RK4IP_OK;
    }
    *count = plan->prof_n[group][pass];
    *mean_ms = *count ? plan->prof_ms[group][pass] / (double)*count : 0.0;
    return RK4IP_OK;
}

int rk4ip_debug_philox(uint64_t seed, const uint32_t* ctr, int64_t n, uint32_t* out, void* stream) {
    if (!ctr || !out || n < 0) return RK4IP_ERR_INVALID_ARG;
    hipError_t e = rk4ip::launch_philox((uint32_t)seed, (uint32_t)(seed >> 32), ctr, n, out,
                                        static_cast<hipStream_t>(stream));
    return e == hipSuccess ? RK4IP_OK : RK4IP_ERR_HIP;
}

int rk4ip_debug_noise(rk4ip_plan_t plan, int group, int64_t step, void* xi) {
    if (!plan || !xi || step < 0 || group < 0 || group >= (int)plan->groups.size()) return RK4IP_ERR_INVALID_ARG;
    HIPCHK(plan, rk4ip::launch_noise(plan->groups[group].d, step, static_cast<float2*>(xi), plan->stream));
    return RK4IP_OK;
}

int rk4ip_debug_fft(rk4ip_plan_t plan, int group, int axis, const void* in, void* out, int64_t nlines, int sign) {
    if (!plan || !in || !out || nlines < 0 || (sign != -1 && sign != 1)) return RK4IP_ERR_INVALID_ARG;
    if (group < 0 || group >= (int)plan->groups.size()) return RK4IP_ERR_INVALID_ARG;
    const GroupHost& g = plan->groups[group];
    if (axis < 0 || axis >= g.p.ndim || g.p.basis) return RK4IP_ERR_INVALID_ARG;
    HIPCHK(plan, rk4ip::launch_fft_lines(static_cast<const float2*>(in), static_cast<float2*>(out), g.p.n[axis], nlines,
                                         sign, g.d.tw[axis], plan->stream));
    return RK4IP_OK;
}

int rk4ip_debug_apply_D(rk4ip_plan_t plan, void* psi, int adjoint) {
    if (!plan || !psi || has_basis_group(plan)) return RK4IP_ERR_INVALID_ARG;
    rk4ip::PassArgs pa{};
    pa.psi = static_cast<float2*>(psi);
    pa.adj = adjoint ? 1 : 0;
    for (auto& g : plan->groups)
        for (int a = 0; a < g.p.ndim; a++) {
            if (plan->f64) {
                Sched sc;
                if (!default_f64_sched(g, a, rk4ip::PASS_D1, &sc)) return RK4IP_ERR_UNSUPPORTED_SHAPE;
                pa.f64 = 1;
                pa.lines = sc.lines;
                pa.seq = sc.seq;
                pa.radix = sc.radix;
            }
            HIPCHK(plan, rk4ip::launch_axis(g.d, a, rk4ip::PASS_D1, pa, plan->stream));
        }
    return RK4IP_OK;
}

int rk4ip_step_noalloc(const rk4ip_problem* probs, int nprob, void* psi_v, int64_t step_index, void* stream_v) {
    if (!psi_v || step_index < 0) return RK4IP_ERR_INVALID_ARG;
    int rc = validate(probs, nprob, 0);
    if (rc != RK4IP_OK) return rc;
    if (nprob > kNoallocMaxGroups) return RK4IP_ERR_INVALID_ARG;
    for (int i = 0; i < nprob; i++)
        if (probs[i].conv_K) return RK4IP_ERR_INVALID_ARG;  // its table is a host-side DFT
    GroupHost gh[kNoallocMaxGroups];
    const Layout L = layout(probs, nprob, 0, gh);
    if (L.total > kNoallocBytes) return RK4IP_ERR_WORKSPACE_TOO_SMALL;
    char* ws = nullptr;
    if ((rc = noalloc_scratch(&ws)) != RK4IP_OK) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream_v);
    float2* psi = static_cast<float2*>(psi_v);
    float2* A = reinterpret_cast<float2*>(ws + L.fields);
    float2* B = A + L.points;
    int64_t offset = 0;
    for (int i = 0; i < nprob; i++) {
        GroupHost& g = gh[i];
        g.p = probs[i];
        fill_group(g, ws, 0, offset);
        offset += g.p.batch * g.M;
        if (g.dct) {
            const int n = (int)g.p.n[0];
            hipLaunchKernelGGL(k_noalloc_basis_tables, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                               const_cast<double2*>(g.d.pairT1), const_cast<float2*>(g.d.tw[0]),
                               const_cast<double2*>(g.d.pairT2), n, kPi / (g.p.hi[0] - g.p.lo[0]), g.p.alpha, g.p.dt,
                               g.p.gamma, g.p.basis);
            if (hipGetLastError() != hipSuccess) return RK4IP_ERR_HIP;
            continue;
        }
        const rk4ip_problem q = transform_problem(g.p, 0);
        for (int a = 0; a < g.p.ndim; a++) {
            const int n = (int)q.n[a];
            hipLaunchKernelGGL(k_noalloc_tables, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                               const_cast<float2*>(g.d.E[a]), const_cast<float2*>(g.d.tw[a]),
                               g.kline ? const_cast<float2*>(g.d.E2) : nullptr, n, 2.0 * kPi / (q.hi[a] - q.lo[a]),
                               q.alpha, q.dt, a == 0 ? q.gamma : 0.0);
            if (hipGetLastError() != hipSuccess) return RK4IP_ERR_HIP;
        }
    }
    // one step of every group with the default schedules: the launches rk4ip_step makes on
    // a plan built without flags
    for (int i = 0; i < nprob; i++) {
        const GroupHost& g = gh[i];
        if (g.p.ndim == 1) {
            if (rk4ip::launch_line_step(g.d, psi, 1, step_index, nullptr, false, 0, false, st, 0) != hipSuccess)
                return RK4IP_ERR_HIP;
            continue;
        }
        PassDef defs[kMaxPasses];
        const int np = pass_list(g.p.ndim, false, defs);
        for (int role : {ROLE_OPEN, ROLE_MID, ROLE_CLOSE}) {
            for (int k = 0; k < np; k++) {
                if (defs[k].role != role) continue;
                rk4ip::PassArgs pa{};
                pa.psi = psi;
                pa.A = A;
                pa.B = B;
                pa.step_off = step_index;
                pa.twice = defs[k].twice;
                if (rk4ip::launch_axis(g.d, defs[k].axis, defs[k].mode, pa, st) != hipSuccess) return RK4IP_ERR_HIP;
            }
        }
    }
    return RK4IP_OK;
}

}  // extern "C"
