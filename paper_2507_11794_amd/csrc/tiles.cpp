// Host construction of the temporally blocked tile plan (see TileMeta in cloth_internal.h):
// per tile, the K-hop region ordered by hop level and the computed nodes' incidences in
// region-local form.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "cloth_internal.h"
#include "host_common.h"

namespace cloth {

int build_tile_plan(const ClothHost& h, const std::vector<int>& group_off, int tile_nodes, int K,
                    hipStream_t stream, TilePlanDevice* out) {
    const int N = h.n;
    if (tile_nodes < 64 || (tile_nodes & 63) || tile_nodes > (1 << 16))
        return fail(CLOTH_EINVAL, "tile_nodes must be a positive multiple of 64 (<= 65536)");
    if (K < 1 || K > kMaxTileK) return fail(CLOTH_EINVAL, "substeps per launch must be in 1..8");
    // tiles: runs of tile_nodes consecutive slots that never cross a cloth boundary
    std::vector<int> tile_begin, tile_group;
    for (size_t g = 0; g + 1 < group_off.size(); ++g)
        for (int a = group_off[g]; a < group_off[g + 1]; a += tile_nodes) {
            tile_begin.push_back(a);
            tile_group.push_back((int)g);
        }
    const int n_tiles = (int)tile_begin.size();
    tile_begin.push_back(N);
    std::vector<TileMeta> meta(n_tiles);
    std::vector<int> region_slot, comp_deg;
    std::vector<uint2> inc;
    std::vector<int> inc_sid;  // spring id of each incidence entry, -1 for padding
    std::vector<int> stamp(N, -1), local(N, 0);
    std::vector<int> region;
    StreamFence fence{stream};  // the vectors above are the sources of the uploads below
    int rmax = 0;
    auto nbr_at = [&](int p, int r) { return h.nbr[(size_t)h.slice_ptr[p >> 6] + (size_t)r * 64 + (p & 63)]; };
    for (int t = 0; t < n_tiles; ++t) {
        region.clear();
        const int a = tile_begin[t];
        const int b = std::min(a + tile_nodes, group_off[tile_group[t] + 1]);
        for (int p = a; p < b; ++p) {
            stamp[p] = t;
            local[p] = (int)region.size();
            region.push_back(p);
        }
        TileMeta& m = meta[t];
        m.group = tile_group[t];
        m.level[0] = (int)region.size();
        size_t lvl_begin = 0;
        for (int k = 1; k <= K; ++k) {
            const size_t lvl_end = region.size();
            std::vector<int> fresh;
            for (size_t q = lvl_begin; q < lvl_end; ++q) {
                const int p = region[q];
                for (int r = 0; r < h.deg[p]; ++r) {
                    const int j = nbr_at(p, r);
                    if (stamp[j] != t) {
                        stamp[j] = t;
                        fresh.push_back(j);
                    }
                }
            }
            std::sort(fresh.begin(), fresh.end());
            for (int j : fresh) {
                local[j] = (int)region.size();
                region.push_back(j);
            }
            m.level[k] = (int)region.size();
            lvl_begin = lvl_end;
        }
        for (int k = K + 1; k <= kMaxTileK; ++k) m.level[k] = m.level[K];
        const int n_comp = m.level[K - 1];
        int maxdeg = 0;
        for (int u = 0; u < n_comp; ++u) maxdeg = std::max(maxdeg, h.deg[region[u]]);
        m.region_off = (int)region_slot.size();
        m.region_n = (int)region.size();
        m.comp_off = (int)comp_deg.size();
        m.inc_pad = (n_comp + 63) & ~63;
        if (inc.size() > (size_t)0x7fffffff - (size_t)maxdeg * m.inc_pad)
            return fail(CLOTH_ENOMEM, "tile plan too large");
        m.inc_off = (int)inc.size();
        rmax = std::max(rmax, m.region_n);
        region_slot.insert(region_slot.end(), region.begin(), region.end());
        inc.resize(inc.size() + (size_t)maxdeg * m.inc_pad, make_uint2(0u, 0u));
        inc_sid.resize(inc.size(), -1);
        for (int u = 0; u < n_comp; ++u) {
            const int p = region[u];
            comp_deg.push_back(h.deg[p]);
            const size_t base = (size_t)h.slice_ptr[p >> 6] + (p & 63);
            for (int r = 0; r < h.deg[p]; ++r) {
                const size_t q = base + (size_t)r * 64;
                const int j = h.nbr[q];
                const int code = h.inc_spring[q];
                const int sid = code >= 0 ? code : ~code;
                inc[(size_t)m.inc_off + (size_t)r * m.inc_pad + u] =
                    make_uint2((uint32_t)local[j], (uint32_t)h.spring_entry[sid]);
                inc_sid[(size_t)m.inc_off + (size_t)r * m.inc_pad + u] = sid;
            }
        }
    }
    if (tile_lds_bytes(rmax, 64, 0) > 160 * 1024)
        return fail(CLOTH_EINVAL, "tile region too large for LDS; use fewer tile nodes or substeps");
    out->arena.release();
    hipError_t e;
    TileMeta* d_meta;
    int *d_rs, *d_deg;
    uint2* d_inc;
    int* d_sid;
    if ((e = out->arena.alloc(&d_meta, meta.size())) ||
        (e = out->arena.alloc(&d_sid, inc_sid.size() + 1)) ||
        (e = out->arena.alloc(&d_rs, region_slot.size())) ||
        (e = out->arena.alloc(&d_deg, comp_deg.size() + 1)) ||
        (e = out->arena.alloc(&d_inc, inc.size() + 1)))
        return hip_fail(e, "hipMalloc tile plan");
    if ((e = hipMemcpyAsync(d_meta, meta.data(), meta.size() * sizeof(TileMeta),
                            hipMemcpyHostToDevice, stream)) ||
        (e = hipMemcpyAsync(d_rs, region_slot.data(), region_slot.size() * 4,
                            hipMemcpyHostToDevice, stream)) ||
        (comp_deg.size() && (e = hipMemcpyAsync(d_deg, comp_deg.data(), comp_deg.size() * 4,
                                                hipMemcpyHostToDevice, stream))) ||
        (inc.size() && (e = hipMemcpyAsync(d_inc, inc.data(), inc.size() * sizeof(uint2),
                                           hipMemcpyHostToDevice, stream))) ||
        (inc_sid.size() && (e = hipMemcpyAsync(d_sid, inc_sid.data(), inc_sid.size() * 4,
                                               hipMemcpyHostToDevice, stream))) ||
        (e = hipStreamSynchronize(stream)))
        return hip_fail(e, "upload tile plan");
    out->tile_nodes = tile_nodes;
    out->K = K;
    out->view.n_tiles = n_tiles;
    out->view.rmax = rmax;
    out->view.ld = h.ld;
    out->view.meta = d_meta;
    out->view.region_slot = d_rs;
    out->view.comp_deg = d_deg;
    out->view.inc = d_inc;
    out->inc_sid = d_sid;
    out->inc_count = inc.size();
    out->bytes = meta.size() * sizeof(TileMeta) + region_slot.size() * 4 + comp_deg.size() * 4 +
                 inc.size() * sizeof(uint2);
    long long comp = 0;
    for (const auto& m : meta) comp += m.level[K - 1];
    out->computed_per_launch_first = comp;
    out->meta_host = std::move(meta);
    return CLOTH_OK;
}

// Work list of the tile kernel.  GRID: one workgroup per tile, mapped so that each of the 8
// XCDs (workgroups are dealt to them round-robin) owns a contiguous run of tiles -- spatial
// neighbours, whose halos and next-launch reads then stay in one L2.  LPT: n_workgroups
// persistent workgroups, tiles by decreasing cost to the least-loaded workgroup.  RR: tile t
// to workgroup t mod n_workgroups.  Cost of a tile = nodes it computes over K substeps.
int build_schedule(TilePlanDevice* plan, int mode, int n_workgroups, hipStream_t stream) {
    const int n = plan->view.n_tiles;
    const int K = plan->K;
    std::vector<int> items, ptr;
    StreamFence fence{stream};
    if (mode == 0 || n_workgroups <= 0 || n_workgroups >= n) {
        const int q = n >> 3, rem = n & 7;
        items.resize(n);
        ptr.resize(n + 1);
        for (int b = 0; b < n; ++b) {
            const int x = b & 7, j = b >> 3;
            items[b] = x * q + (x < rem ? x : rem) + j;
            ptr[b] = b;
        }
        ptr[n] = n;
    } else {
        const int W = n_workgroups;
        std::vector<std::vector<int>> lists(W);
        if (mode == 1) {
            std::vector<std::pair<long long, int>> cost(n);
            for (int t = 0; t < n; ++t) {
                long long c = 0;
                for (int s = 1; s <= K; ++s) c += plan->meta_host[t].level[K - s];
                cost[t] = {-c, t};
            }
            std::sort(cost.begin(), cost.end());
            std::vector<std::pair<long long, int>> heap;  // (load, workgroup), min-heap
            for (int b = 0; b < W; ++b) heap.emplace_back(0, b);
            auto cmp = [](const std::pair<long long, int>& x, const std::pair<long long, int>& y) {
                return x > y;
            };
            std::make_heap(heap.begin(), heap.end(), cmp);
            for (const auto& ct : cost) {
                std::pop_heap(heap.begin(), heap.end(), cmp);
                auto& top = heap.back();
                lists[top.second].push_back(ct.second);
                top.first += -ct.first;
                std::push_heap(heap.begin(), heap.end(), cmp);
            }
            for (auto& l : lists) std::sort(l.begin(), l.end());
        } else {
            for (int t = 0; t < n; ++t) lists[t % W].push_back(t);
        }
        ptr.push_back(0);
        for (const auto& l : lists) {
            items.insert(items.end(), l.begin(), l.end());
            ptr.push_back((int)items.size());
        }
    }
    plan->sched_arena.release();
    int *d_items, *d_ptr;
    hipError_t e;
    if ((e = plan->sched_arena.alloc(&d_items, items.size() + 1)) ||
        (e = plan->sched_arena.alloc(&d_ptr, ptr.size())) ||
        (e = hipMemcpyAsync(d_items, items.data(), items.size() * 4, hipMemcpyHostToDevice, stream)) ||
        (e = hipMemcpyAsync(d_ptr, ptr.data(), ptr.size() * 4, hipMemcpyHostToDevice, stream)) ||
        (e = hipStreamSynchronize(stream)))
        return hip_fail(e, "upload schedule");
    plan->view.items = d_items;
    plan->view.item_ptr = d_ptr;
    plan->view.n_workgroups = (int)ptr.size() - 1;
    plan->schedule = mode;
    plan->sched_workgroups = n_workgroups;
    return CLOTH_OK;
}

}  // namespace cloth
