// kernels_pass_merged.hip -- one launch of a pass kind over every 2D/3D group of a plan.
//
// Many instances of uneven lattice size (the multi-path and batched runs of Dennis, Hope &
// Johnsson, arXiv:1204.4255, Sec. 4.6) advance together: instead of one launch per group
// and pass, each pass kind is one launch whose workgroups are divided among the groups by
// a work list of block offsets. A workgroup finds its group by a block-uniform search,
// then runs the single-group pass body of pass_common.h on its tile, with the length
// chosen by a block-uniform switch. The schedule is fixed so that every group's tiles have
// the same workgroup size: radix 8, both fields at once, 256 threads, that is 2048/N lines
// or columns per tile, for lengths 128 and 256 (one kernel holding every length's body is
// allocated for the largest; 512 would cost the others occupancy). No workgroup waits
// for another.
#include "pass_common.h"

namespace rk4ip {

template <int N>
constexpr int merged_lines() { return 256 * 8 / N; }

template <int N, int MODE, bool CONTIG>
using MergedLds = AxisLds<N, MODE, CONTIG, merged_lines<N>(), 0, 8, false>;

// Register allocation: four waves per SIMD for the one-transform-pair passes and XF (as
// the per-group kernels' four-wave variants); LF, which holds both stage fields through its
// second transform, keeps three rather than spill.
template <int MODE>
constexpr int merged_occ() { return MODE == PASS_LF ? 1 : 4; }

template <int MODE, bool CONTIG, bool NOISE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(merged_occ<MODE>())))
k_axis_merged(MergedList ml, int axis, PassArgs args) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const uint32_t b = blockIdx.x;
    int k = 0;
    while (k + 1 < ml.count && b >= ml.block0[k + 1]) k++;  // uniform over the workgroup
    const uint32_t bid = b - ml.block0[k];
    const uint32_t nblk = ml.nblk[k];
    if (bid >= nblk) return;  // padding that starts every group on a multiple of 8 blocks
    // the group's parameters, read where used (uniform loads; nothing the pass writes
    // aliases them)
    const GroupDev* __restrict__ gp = ml.groups + ml.gid[k];
    const GroupDev& g = *gp;
    c32* smem = reinterpret_cast<c32*>(smem_raw);
    switch (g.n[axis]) {
        case 128: axis_body<128, MODE, CONTIG, merged_lines<128>(), NOISE, 0, 8, false>(g, axis, args, bid, nblk, smem); break;
        case 256: axis_body<256, MODE, CONTIG, merged_lines<256>(), NOISE, 0, 8, false>(g, axis, args, bid, nblk, smem); break;
        default: break;  // refused at plan time
    }
}

template <int MODE, bool CONTIG>
static size_t merged_lds(int N) {
    switch (N) {
        case 128: return MergedLds<128, MODE, CONTIG>::BYTES;
        case 256: return MergedLds<256, MODE, CONTIG>::BYTES;
        default: return 0;
    }
}

size_t merged_lds_bytes(int N, int mode, int axis) {
    const bool contig = axis == 0;
    switch (mode) {
        case PASS_FIRST: return contig ? merged_lds<PASS_FIRST, true>(N) : 0;
        case PASS_LAST2: return contig ? merged_lds<PASS_LAST2, true>(N) : 0;
        case PASS_XF: return contig ? merged_lds<PASS_XF, true>(N) : 0;
        case PASS_LF: return contig ? 0 : merged_lds<PASS_LF, false>(N);
        case PASS_D2: return contig ? 0 : merged_lds<PASS_D2, false>(N);
        default: return 0;
    }
}

int merged_tile_lines(int N) { return 2048 / N; }

template <int MODE, bool CONTIG>
static hipError_t go_merged(const MergedList& ml, int axis, bool noise, uint32_t blocks, size_t smem, const PassArgs& a,
                            hipStream_t s) {
    if (noise)
        hipLaunchKernelGGL((k_axis_merged<MODE, CONTIG, true>), dim3(blocks), dim3(256), smem, s, ml, axis, a);
    else
        hipLaunchKernelGGL((k_axis_merged<MODE, CONTIG, false>), dim3(blocks), dim3(256), smem, s, ml, axis, a);
    return hipGetLastError();
}

hipError_t launch_axis_merged(const MergedList& ml, int mode, int axis, bool noise, uint32_t blocks, size_t smem,
                              const PassArgs& a, hipStream_t s) {
    if (blocks == 0) return hipSuccess;
    const bool contig = axis == 0;
    switch (mode) {
        case PASS_FIRST: return contig ? go_merged<PASS_FIRST, true>(ml, axis, noise, blocks, smem, a, s) : hipErrorInvalidValue;
        case PASS_LAST2: return contig ? go_merged<PASS_LAST2, true>(ml, axis, noise, blocks, smem, a, s) : hipErrorInvalidValue;
        case PASS_XF: return contig ? go_merged<PASS_XF, true>(ml, axis, noise, blocks, smem, a, s) : hipErrorInvalidValue;
        case PASS_LF: return contig ? hipErrorInvalidValue : go_merged<PASS_LF, false>(ml, axis, noise, blocks, smem, a, s);
        case PASS_D2: return contig ? hipErrorInvalidValue : go_merged<PASS_D2, false>(ml, axis, noise, blocks, smem, a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace rk4ip
