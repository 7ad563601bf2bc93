// Second pass of the one-substep kernel for nodes whose grid cell lists many references.
// A node's collision query is a chain of dependent loads (reference boxes, then the box hits'
// geometry) whose length grows with its cell's reference count; the wavefronts holding such
// nodes set the substep's length.  The first pass integrates every node, resolves the light
// ones and lists the heavy ones (their predicted state is already written).  Here four
// lanes share one heavy node: lane j tests the j-th quarter of the cell's references, lists
// its box hits in LDS, runs the narrow phase on them and records each contact's push and
// normal; the node's first lane then sums the four lanes' contacts in order.  The quarters
// are consecutive and each lane keeps its own order, so the contacts are summed in
// ascending triangle id with the same operations as the one-lane query: the result is
// identical bit for bit.
#include <algorithm>

#include "cloth_device.h"
#include "cloth_internal.h"

namespace cloth {

namespace {

constexpr int kLanes = 4;
constexpr int kPartHits = 24;      // box hits one lane lists
constexpr int kPartContacts = 8;   // contacts one lane records
constexpr size_t kWaveLds = (size_t)kPartHits * 64 * 4 + (size_t)kPartContacts * 64 * 16;

template <bool GROUPED>
__global__ void __launch_bounds__(256)
    k_heavy(const ClothView cv, const StepParams sp, int* __restrict__ heavy, const int parity,
            float* __restrict__ xd, float* __restrict__ vd, const SurfaceView* __restrict__ svs,
            const int* __restrict__ node_group) {
    extern __shared__ uint32_t heavy_lds[];
    const int count = min(heavy[parity], cv.n);  // never past the list, whatever the counter
    // the other parity's list is refilled by the next substep's first pass
    if (blockIdx.x == 0 && threadIdx.x == 0) heavy[parity ^ 1] = 0;
    const int* nodes = heavy + kHeavyListOff + (size_t)parity * cv.ld;
    const int lane = threadIdx.x & 63, part = threadIdx.x % kLanes;
    const int base = lane & ~(kLanes - 1);
    uint32_t* list = heavy_lds + (threadIdx.x >> 6) * (kWaveLds / 4) + lane;
    float4* rec = reinterpret_cast<float4*>(heavy_lds + (threadIdx.x >> 6) * (kWaveLds / 4) +
                                            kPartHits * 64) + lane;
    const int ld = cv.ld;
    constexpr int kNodesPerBlock = 256 / kLanes;
    // the loop bounds are uniform over the grid, so every lane takes part in the shuffles
    for (int c0 = blockIdx.x * kNodesPerBlock; c0 < count; c0 += gridDim.x * kNodesPerBlock) {
        const int slot = c0 + threadIdx.x / kLanes;
        const bool act = slot < count;
        const int i = act ? nodes[slot] : 0;
        float px = 0.0f, py = 0.0f, pz = 0.0f, qx = 0.0f, qy = 0.0f, qz = 0.0f;
        SurfaceView sv{};
        int nc = 0, overflow = 0;
        if (act) {
            px = xd[i];
            py = xd[ld + i];
            pz = xd[2 * ld + i];
            qx = vd[i];
            qy = vd[ld + i];
            qz = vd[2 * ld + i];
            sv = svs[GROUPED ? node_group[i] : 0];
            const int cell = cell_of(sv, px, py, pz);  // inside the grid: the first pass checked
            const gptr<uint32_t> cs = gmem(sv.cell_start);
            const uint32_t b = cs[cell], e = cs[cell + 1];
            const uint32_t q = (e - b + kLanes - 1) / kLanes;
            const uint32_t r0 = min(e, b + part * q), r1 = min(e, r0 + q);
            int nh = 0;
            for (uint32_t r = r0; r < r1; r += kRefRound) {
                float4 lo[kRefRound], hi[kRefRound];
#pragma unroll
                for (int k = 0; k < kRefRound; ++k) {
                    lo[k] = ldg4(sv.ref_lo, r + k);
                    hi[k] = ldg4(sv.ref_hi, r + k);
                }
#pragma unroll
                for (int k = 0; k < kRefRound; ++k)
                    if (r + k < r1 && in_box(lo[k], hi[k], px, py, pz)) {
                        if (nh < kPartHits) list[nh * 64] = (uint32_t)__float_as_int(lo[k].w);
                        ++nh;
                    }
            }
            overflow = nh > kPartHits;
            const float th = sv.thickness;
            auto record = [&](const float4& n, float s, uint32_t) {
                if (nc < kPartContacts) rec[nc * 64] = make_float4(th - s, n.x, n.y, n.z);
                ++nc;
            };
            for (int h0 = 0; h0 < nh && !overflow; h0 += 8) {
                uint32_t tt[8];
                float4 g[8][3];
#pragma unroll
                for (int k = 0; k < 8; ++k) tt[k] = list[min(h0 + k, nh - 1) * 64];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    g[k][0] = ldg4(sv.geo, 3 * (size_t)tt[k]);
                    g[k][1] = ldg4(sv.geo, 3 * (size_t)tt[k] + 1);
                    g[k][2] = ldg4(sv.geo, 3 * (size_t)tt[k] + 2);
                }
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    if (h0 + k < nh)
                        narrow_visit(sv, tt[k], g[k][0], g[k][1], g[k][2], px, py, pz, record);
            }
            overflow |= nc > kPartContacts;
        }
        // the node's first lane gathers its group's counts
        int ncs[kLanes];
        int ovf = 0;
#pragma unroll
        for (int j = 0; j < kLanes; ++j) {
            ncs[j] = __shfl(nc, base + j);
            ovf |= __shfl(overflow, base + j);
        }
        if (act && part == 0) {
            if (ovf) {
                collide(sv, sp.restitution, px, py, pz, qx, qy, qz);  // the one-lane query
            } else {
                float sx = 0.0f, sy = 0.0f, sz = 0.0f;
                int contacts = 0;
                const float4* group = reinterpret_cast<const float4*>(rec) - lane + base;
#pragma unroll
                for (int j = 0; j < kLanes; ++j)
                    for (int k = 0; k < ncs[j]; ++k) {
                        const float4 cr = group[k * 64 + j];
                        sx += cr.x * cr.y;
                        sy += cr.x * cr.z;
                        sz += cr.x * cr.w;
                        ++contacts;
                    }
                respond(contacts, sx, sy, sz, sp.restitution, px, py, pz, qx, qy, qz);
            }
            xd[i] = px;
            xd[ld + i] = py;
            xd[2 * ld + i] = pz;
            vd[i] = qx;
            vd[ld + i] = qy;
            vd[2 * ld + i] = qz;
            if (sp.check_nan) {
                const float sum = px + py + pz + qx + qy + qz;
                if (!__builtin_isfinite(sum)) atomicOr(sp.nan_flag, 1);
            }
        }
    }
}

}  // namespace

size_t heavy_lds_bytes() { return 4 * kWaveLds; }

hipError_t launch_heavy(const ClothView& cv, const StepParams& sp, int* heavy, int parity,
                        float* xd, float* vd, const SurfaceView* svs, const int* node_group,
                        hipStream_t st) {
    if (cv.n <= 0) return hipSuccess;
    // persistent grid: two workgroups per compute unit loop over the listed nodes
    const int nodes_per_block = 256 / kLanes;
    const int grid = (int)std::min<long long>(512, ((long long)cv.n + nodes_per_block - 1) / nodes_per_block);
    if (node_group)
        k_heavy<true><<<grid, 256, heavy_lds_bytes(), st>>>(cv, sp, heavy, parity, xd, vd, svs,
                                                            node_group);
    else
        k_heavy<false><<<grid, 256, heavy_lds_bytes(), st>>>(cv, sp, heavy, parity, xd, vd, svs,
                                                             nullptr);
    return hipGetLastError();
}

}  // namespace cloth
