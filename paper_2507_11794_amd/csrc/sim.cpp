// The plain and batch C ABI (include/cloth.h): create / step / state access / launch
// configuration, and the substep scheduler (tile plans, schedules, hipGraph replay).  A batch
// of independent cloths of uneven sizes (cloth_batch_*) is one simulation handle holding
// every cloth: one node array, tiles that never cross two cloths, one surface grid per cloth,
// and one graph of launches for all of them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "sim.h"

namespace cloth {

int check_launch(const cloth_launch& c) {
    if (c.kernel < CLOTH_KERNEL_TILE || c.kernel > CLOTH_KERNEL_GRID)
        return fail(CLOTH_EINVAL, "unknown kernel");
    if (c.block_threads < 64 || c.block_threads > 256 || (c.block_threads & 63))
        return fail(CLOTH_EINVAL, "block_threads must be 64, 128, 192 or 256");
    if (c.hit_slots < 0 || c.hit_slots > kMaxHitSlots)
        return fail(CLOTH_EINVAL, "hit_slots must be in 0..64");
    if (c.split_refs < 0) return fail(CLOTH_EINVAL, "split_refs must be >= 0");
    if (c.xcd_runs < 0 || c.xcd_runs > kMaxXcdRuns)
        return fail(CLOTH_EINVAL, "xcd_runs must be in 0..4096");
    if (c.kernel == CLOTH_KERNEL_TILE) {
        if (c.tile_nodes < 64 || c.tile_nodes > 4096 || (c.tile_nodes & 63))
            return fail(CLOTH_EINVAL, "tile_nodes must be a multiple of 64 in 64..4096");
        if (c.substeps_per_launch < 1 || c.substeps_per_launch > kMaxTileK)
            return fail(CLOTH_EINVAL, "substeps_per_launch must be in 1..8");
        if (c.schedule < CLOTH_SCHED_GRID || c.schedule > CLOTH_SCHED_RR)
            return fail(CLOTH_EINVAL, "unknown schedule");
        if (c.schedule != CLOTH_SCHED_GRID && (c.workgroups < 1 || c.workgroups > (1 << 20)))
            return fail(CLOTH_EINVAL, "persistent schedules need 1..2^20 workgroups");
    }
    return CLOTH_OK;
}

int ensure_plan(cloth_sim* s, const cloth_launch& c) {
    if (c.kernel != CLOTH_KERNEL_TILE) return CLOTH_OK;
    const bool plan_ok = s->plan.tile_nodes == c.tile_nodes && s->plan.K == c.substeps_per_launch;
    const int wg = c.schedule == CLOTH_SCHED_GRID ? 0 : c.workgroups;
    const bool sched_ok = plan_ok && s->plan.schedule == c.schedule && s->plan.sched_workgroups == wg;
    if (sched_ok) return CLOTH_OK;
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "synchronise before replanning");
    s->drop_graphs();
    if (!plan_ok) {
        TilePlanDevice fresh;
        int st = build_tile_plan(s->host, s->group_off, c.tile_nodes, c.substeps_per_launch,
                                 s->stream, &fresh);
        if (st != CLOTH_OK) return st;
        s->plan.arena.release();
        s->plan.arena.ptrs.swap(fresh.arena.ptrs);
        s->plan.meta_host.swap(fresh.meta_host);
        s->plan.tile_nodes = fresh.tile_nodes;
        s->plan.K = fresh.K;
        s->plan.view = fresh.view;
        s->plan.view.w = s->dev.w;
        s->plan.view.ptab = s->dev.ptab;
        s->plan.view.svs = s->svs_dev;
        s->plan.inc_sid = fresh.inc_sid;
        s->plan.inc_count = fresh.inc_count;
        s->plan.bytes = fresh.bytes;
        s->plan.computed_per_launch_first = fresh.computed_per_launch_first;
        s->plan.schedule = -1;
    }
    int st = build_schedule(&s->plan, c.schedule, wg, s->stream);
    if (st != CLOTH_OK) return st;
    ++s->plan_version;
    return CLOTH_OK;
}

int ensure_springs(cloth_sim* s) {
    if (s->springs.ready) return CLOTH_OK;
    const int S = s->n_springs;
    const size_t ld = (size_t)s->dev.ld;
    // ends as internal slots; parameters from the handle's per-spring copies
    const std::vector<float>& rest = s->rest;
    std::vector<int> perm(S);
    for (int q = 0; q < S; ++q) perm[q] = q;
    auto lo = [&](int q) { return std::min(s->host.slot[s->ends[2 * q]], s->host.slot[s->ends[2 * q + 1]]); };
    auto hi = [&](int q) { return std::max(s->host.slot[s->ends[2 * q]], s->host.slot[s->ends[2 * q + 1]]); };
    std::sort(perm.begin(), perm.end(), [&](int p, int q) {
        return lo(p) != lo(q) ? lo(p) < lo(q) : (hi(p) != hi(q) ? hi(p) < hi(q) : p < q);
    });
    std::vector<int> a(S), b(S);
    std::vector<float> k(S), c(S), L0(S);
    StreamFence fence{s->stream};
    for (int r = 0; r < S; ++r) {
        const int q = perm[r];
        a[r] = s->host.slot[s->ends[2 * q]];
        b[r] = s->host.slot[s->ends[2 * q + 1]];
        k[r] = s->k[q];
        c[r] = s->c[q];
        L0[r] = rest[q];
    }
    SpringDevice& d = s->springs;
    d.arena.release();
    int *da = nullptr, *db = nullptr, *sid = nullptr;
    float *dk = nullptr, *dc = nullptr, *dl = nullptr, *F = nullptr;
    hipError_t e;
    if ((e = d.arena.alloc(&da, (size_t)S)) || (e = d.arena.alloc(&db, (size_t)S)) ||
        (e = d.arena.alloc(&sid, (size_t)S)) || (e = d.arena.alloc(&dk, (size_t)S)) ||
        (e = d.arena.alloc(&dc, (size_t)S)) || (e = d.arena.alloc(&dl, (size_t)S)) ||
        (e = d.arena.alloc(&F, 3 * ld)) ||
        (e = hipMemcpyAsync(da, a.data(), 4 * (size_t)S, hipMemcpyHostToDevice, s->stream)) ||
        (e = hipMemcpyAsync(db, b.data(), 4 * (size_t)S, hipMemcpyHostToDevice, s->stream)) ||
        (e = hipMemcpyAsync(sid, perm.data(), 4 * (size_t)S, hipMemcpyHostToDevice, s->stream)) ||
        (e = hipMemcpyAsync(dk, k.data(), 4 * (size_t)S, hipMemcpyHostToDevice, s->stream)) ||
        (e = hipMemcpyAsync(dc, c.data(), 4 * (size_t)S, hipMemcpyHostToDevice, s->stream)) ||
        (e = hipMemcpyAsync(dl, L0.data(), 4 * (size_t)S, hipMemcpyHostToDevice, s->stream)) ||
        (e = hipMemsetAsync(F, 0, 12 * ld, s->stream)) || (e = hipStreamSynchronize(s->stream))) {
        d.arena.release();
        return hip_fail(e, "spring list");
    }
    d.view = SpringList{S, da, db, dk, dc, dl};
    d.sid = sid;
    d.k = dk;
    d.c = dc;
    d.F = F;
    d.ready = true;
    return CLOTH_OK;
}

int set_launch(cloth_sim* s, const cloth_launch& cfg) {
    int st = check_launch(cfg);
    if (st != CLOTH_OK) return st;
    if (cfg.kernel == CLOTH_KERNEL_GRID && !s->dev.sten_code)
        return fail(CLOTH_EINVAL, "the grid kernel needs grid cloths whose springs join nodes at "
                                  "most two rows or columns apart (the stencil), one per offset");
    // until this call succeeds the plan may not match s->launch; the next run re-applies it
    s->launch_ready = false;
    if ((st = ensure_plan(s, cfg)) != CLOTH_OK) return st;
    // dynamic LDS of the chosen kernel: check it fits and raise the kernels' limit
    const int slots = s->any_collision ? cfg.hit_slots : 0;
    const bool lanes_kernel = cfg.kernel == CLOTH_KERNEL_LANES2 || cfg.kernel == CLOTH_KERNEL_LANES4;
    const size_t lds = cfg.kernel == CLOTH_KERNEL_TILE
                           ? tile_lds_bytes(s->plan.view.rmax, cfg.block_threads, slots)
                       : lanes_kernel ? (s->any_collision ? lanes_lds_bytes(cfg.block_threads, slots) : 0)
                       : cfg.kernel == CLOTH_KERNEL_GRID ? grid_lds_bytes(slots)
                                      : (size_t)(cfg.block_threads / 64) * wave_query_lds(slots);
    if (lds > 160 * 1024)
        return fail(CLOTH_EINVAL, "tile region plus hit lists exceed 160 KiB of LDS");
    const bool scatter = cfg.kernel == CLOTH_KERNEL_SCATTER_F32 || cfg.kernel == CLOTH_KERNEL_SCATTER_FIX;
    if (scatter && (st = ensure_springs(s)) != CLOTH_OK) return st;
    if (cfg.kernel == CLOTH_KERNEL_DIRECT && cfg.split_refs > 0) {
        // the second pass's node lists; both counters start at zero
        hipError_t e = hipSuccess;
        if (!s->heavy_dev) e = s->arena.alloc(&s->heavy_dev, heavy_words(s->dev.ld));
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e == hipSuccess) e = hipMemsetAsync(s->heavy_dev, 0, 2 * sizeof(int), s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return hip_fail(e, "second-pass lists");
    }
    hipError_t pe = cfg.kernel == CLOTH_KERNEL_TILE ? prepare_tile_kernels(lds)
                    : scatter                       ? prepare_scatter_kernels(lds)
                    : lanes_kernel                  ? prepare_lanes_kernels(lds)
                    : cfg.kernel == CLOTH_KERNEL_GRID ? prepare_grid_kernels(lds)
                                                    : prepare_substep_kernels(lds);
    if (pe != hipSuccess) return hip_fail(pe, "kernel LDS attribute");
    cloth_launch norm = cfg;
    if (cfg.kernel != CLOTH_KERNEL_TILE) {
        norm.schedule = CLOTH_SCHED_GRID;
        norm.workgroups = 0;
    }
    // grid kernel: one wavefront per tile, or two (128 threads and more ask for two)
    if (cfg.kernel == CLOTH_KERNEL_GRID) norm.block_threads = cfg.block_threads >= 128 ? 128 : 64;
    if (cfg.kernel != CLOTH_KERNEL_DIRECT) norm.split_refs = 0;
    if (std::memcmp(&norm, &s->launch, sizeof(cloth_launch)) != 0) {
        // captured graphs hold the old configuration's kernels and arguments
        hipError_t e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return hip_fail(e, "synchronise");
        s->drop_graphs();
    }
    s->launch = norm;
    s->launch_ready = true;
    return CLOTH_OK;
}

namespace {

// One launch advancing K substeps from buffer `src` into buffer `src ^ 1`.
hipError_t launch_once(cloth_sim* s, const StepParams& sp, int K, int src, hipStream_t st) {
    const int dst = src ^ 1;
    if (s->mt && s->any_collision)
        return launch_mt_substep(s->dev.view(), sp,
                                 MtTopology{s->order_dev, s->slot_dev,
                                            s->groups.size() > 1 ? s->node_group_dev : nullptr,
                                            s->group_desc_dev},
                                 s->svs_dev, s->dev.x[src], s->dev.v[src], s->mt_pred,
                                 s->dev.x[dst], s->dev.v[dst], s->launch.block_threads, st);
    if (s->launch.kernel == CLOTH_KERNEL_TILE && (K < 1 || K > s->plan.K))
        return hipErrorInvalidValue;  // the plan covers at most plan.K substeps per launch
    if (s->launch.kernel == CLOTH_KERNEL_TILE)
        return launch_tiles(s->plan.view, K, s->any_collision, sp, s->dev.x[src], s->dev.v[src],
                            s->dev.x[dst], s->dev.v[dst], s->launch.block_threads,
                            s->launch.hit_slots, st);
    if (s->launch.kernel == CLOTH_KERNEL_SCATTER_F32 || s->launch.kernel == CLOTH_KERNEL_SCATTER_FIX)
        return launch_scatter_substep(s->dev.view(), s->springs.view,
                                      s->launch.kernel == CLOTH_KERNEL_SCATTER_FIX,
                                      s->any_collision, sp, s->springs.F, s->dev.x[src],
                                      s->dev.v[src], s->dev.x[dst], s->dev.v[dst],
                                      s->launch.block_threads, st, s->svs_dev,
                                      s->groups.size() > 1 ? s->node_group_dev : nullptr,
                                      s->launch.hit_slots, s->launch.xcd_runs);
    if (s->launch.kernel == CLOTH_KERNEL_GRID)
        return launch_grid_substep(
            s->dev.view(), s->dev.grid_view(),
            s->groups.size() == 1 ? s->surfs[0].view.n_tris > 0 : s->any_collision, sp,
            s->dev.x[src], s->dev.v[src], s->dev.x[dst], s->dev.v[dst], st, s->svs_dev,
            s->groups.size() > 1, s->launch.hit_slots, s->launch.xcd_runs,
            s->launch.block_threads / 64);
    if (s->launch.kernel == CLOTH_KERNEL_LANES2 || s->launch.kernel == CLOTH_KERNEL_LANES4)
        return launch_substep_lanes(
            s->launch.kernel == CLOTH_KERNEL_LANES2 ? 2 : 4, s->dev.view(),
            s->groups.size() == 1 ? s->surfs[0].view.n_tris > 0 : s->any_collision, sp,
            s->dev.x[src], s->dev.v[src], s->dev.x[dst], s->dev.v[dst], s->launch.block_threads,
            st, s->svs_dev, s->groups.size() > 1 ? s->node_group_dev : nullptr,
            s->launch.hit_slots, s->launch.xcd_runs);
    if (s->groups.size() == 1)
        return launch_substep(s->dev.view(), s->surfs[0].view.n_tris > 0, sp, s->dev.x[src],
                              s->dev.v[src], s->dev.x[dst], s->dev.v[dst], s->launch.block_threads,
                              st, s->svs_dev, nullptr, s->launch.hit_slots,
                              s->launch.xcd_runs, s->launch.split_refs, s->heavy_dev, src);
    return launch_substep(s->dev.view(), s->any_collision, sp, s->dev.x[src], s->dev.v[src],
                          s->dev.x[dst], s->dev.v[dst], s->launch.block_threads, st, s->svs_dev,
                          s->node_group_dev, s->launch.hit_slots, s->launch.xcd_runs,
                          s->launch.split_refs, s->heavy_dev, src);
}

// A captured graph of `chunk` launches of K substeps starting from buffer `parity` (an odd
// chunk ends on the other buffer).
hipGraphExec_t get_graph(cloth_sim* s, const StepParams& sp, int K, int chunk, int parity) {
    unsigned hb;
    std::memcpy(&hb, &sp.h, 4);
    for (auto& g : s->graphs)
        if (g.h_bits == hb && g.K == K && g.chunk == chunk && g.parity == parity &&
            g.plan_version == s->plan_version)
            return g.exec;
    if (!s->capture && hipStreamCreateWithFlags(&s->capture, hipStreamNonBlocking) != hipSuccess) {
        s->capture = nullptr;
        return nullptr;
    }
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(s->capture, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return nullptr;
    bool ok = true;
    int cur = parity;
    for (int i = 0; i < chunk; ++i) {
        if (launch_once(s, sp, K, cur, s->capture) != hipSuccess) ok = false;
        cur ^= 1;
    }
    if (hipStreamEndCapture(s->capture, &graph) != hipSuccess || !ok || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        return nullptr;
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (s->graphs.size() >= 8) {
        // the oldest graph may still run on the stream: let it finish first
        (void)hipStreamSynchronize(s->stream);
        (void)hipGraphExecDestroy(s->graphs.front().exec);
        s->graphs.erase(s->graphs.begin());
    }
    s->graphs.push_back(GraphEntry{hb, K, chunk, parity, s->plan_version, exec});
    return exec;
}

}  // namespace

// Any split of the substeps into launches gives the same bits, so the schedule only affects
// speed.
int run_substeps(cloth_sim* s, float h, long long total) {
    StepParams sp;
    sp.h = h;
    for (int q = 0; q < 3; ++q) sp.g[q] = s->p.gravity[q];
    sp.restitution = s->p.restitution;
    sp.check_nan = (s->p.flags & CLOTH_F_CHECK_NAN) ? 1 : 0;
    sp.nan_flag = s->nan_flag;
    sp.fext = s->fext_on ? s->fext_dev : nullptr;
    sp.fext_ld = s->dev.ld;
    int st = CLOTH_OK;
    if (!s->launch_ready) {
        if ((st = set_launch(s, s->launch)) != CLOTH_OK) return st;
        s->launch_ready = true;
    }
    s->roll.ready = false;  // stepping moves the state away from a rollout's checkpoints
    const int K = substeps_per_launch(s);
    long long launches = total / K;
    const int rem = (int)(total % K);
    if (s->launch.use_graph) {
        // about 32 substeps per graph, an even number of launches so the buffers return to
        // their starting parity after every replay
        int chunk = std::max(1, 32 / K);
        chunk += chunk & 1;
        if (launches >= chunk) {
            hipGraphExec_t exec = get_graph(s, sp, K, chunk, s->dev.cur);
            if (exec) {
                for (long long r = launches / chunk; r > 0; --r) {
                    hipError_t e = hipGraphLaunch(exec, s->stream);
                    if (e != hipSuccess) return hip_fail(e, "graph launch");
                }
                launches %= chunk;
            }
        }
        // the remainder (two or more launches) as one graph of its own length, so a call of
        // any length replays graphs only once its graphs exist
        if (launches >= 2) {
            hipGraphExec_t exec = get_graph(s, sp, K, (int)launches, s->dev.cur);
            if (exec) {
                hipError_t e = hipGraphLaunch(exec, s->stream);
                if (e != hipSuccess) return hip_fail(e, "graph launch");
                s->dev.cur ^= (int)(launches & 1);
                launches = 0;
            }
        }
    }
    for (long long i = 0; i < launches; ++i) {
        hipError_t e = launch_once(s, sp, K, s->dev.cur, s->stream);
        if (e != hipSuccess) return hip_fail(e, "substep launch");
        s->dev.cur ^= 1;
    }
    if (rem) {
        hipError_t e = launch_once(s, sp, rem, s->dev.cur, s->stream);
        if (e != hipSuccess) return hip_fail(e, "substep launch");
        s->dev.cur ^= 1;
    }
    return CLOTH_OK;
}

int step_sim(cloth_sim* s, float dt, int n_substeps, int n_steps) {
    if (s->surface_broken)
        return fail(CLOTH_ESTATE, "a surface update failed; the handle cannot step until one succeeds");
    if (!(dt > 0.0f) || !std::isfinite(dt)) return fail(CLOTH_EINVAL, "dt must be positive and finite");
    if (n_substeps < 1 || n_steps < 0) return fail(CLOTH_EINVAL, "n_substeps >= 1 and n_steps >= 0");
    const float h = dt / (float)n_substeps;
    if (!(s->p.flags & CLOTH_F_NO_STABILITY_CHECK))
        for (size_t g = 0; g < s->groups.size(); ++g)
            if (unstable(s->groups[g].omega2, s->groups[g].gamma, h))
                return fail(CLOTH_EUNSTABLE,
                            "cloth " + std::to_string(g) + ": substep h = " + std::to_string(h) +
                                " s exceeds the explicit stability bound (omega^2 = " +
                                std::to_string(s->groups[g].omega2) + ", gamma = " +
                                std::to_string(s->groups[g].gamma) + "); use more substeps");
    return run_substeps(s, h, (long long)n_steps * n_substeps);
}

void refresh_stability(cloth_sim* s) {
    for (auto& g : s->groups) {
        ClothHostInput in{};
        in.nx = g.n;
        in.ny = 1;
        in.x0 = s->x0.data() + 3 * (size_t)g.node_off;
        in.mass = s->mass.data() + g.node_off;
        in.pinned = s->pinned.data() + g.node_off;
        in.n_springs = 0;
        // springs of this cloth, renumbered to the cloth's own node ids
        std::vector<int> ends(2 * (size_t)g.n_springs);
        for (int q = 0; q < 2 * g.n_springs; ++q)
            ends[q] = s->ends[2 * (size_t)g.spring_off + q] - g.node_off;
        in.n_springs = g.n_springs;
        in.ends = ends.data();
        in.k = s->k.data() + g.spring_off;
        in.c = s->c.data() + g.spring_off;
        stability_bounds(in, &g.omega2, &g.gamma);
    }
}

int read_state_range(const cloth_sim* s, int group, float* x_out, float* v_out) {
    const GroupInfo& g = s->groups[group];
    const size_t ld = (size_t)s->dev.ld, n = (size_t)g.n;
    hipError_t e;
    if (!s->export_dev) {
        size_t most = 1;
        for (const GroupInfo& q : s->groups) most = std::max(most, (size_t)q.n);
        if ((e = hipMalloc((void**)&s->export_dev, 24 * most)))
            return hip_fail(e, "read state staging");
        if ((e = hipHostMalloc((void**)&s->export_host, 24 * most + 4, hipHostMallocDefault))) {
            (void)hipFree(s->export_dev);
            s->export_dev = nullptr;
            s->export_host = nullptr;
            return hip_fail(e, "read state staging");
        }
    }
    // AoS in node-id order on the device (slot_dev maps node id -> internal slot), then one
    // copy of x (and v) and the status flag into pinned memory
    const int* slot = s->slot_dev + g.node_off;
    const size_t nv = v_out ? 2 : 1;
    if ((e = launch_export((int)n, (int)ld, slot, s->dev.x[s->dev.cur], s->export_dev, s->stream)) ||
        (v_out && (e = launch_export((int)n, (int)ld, slot, s->dev.v[s->dev.cur],
                                     s->export_dev + 3 * n, s->stream))) ||
        (e = hipMemcpyAsync(s->export_host, s->export_dev, 12 * n * nv, hipMemcpyDeviceToHost,
                            s->stream)) ||
        (e = hipMemcpyAsync(s->export_host + 6 * n, s->nan_flag, 4, hipMemcpyDeviceToHost,
                            s->stream)) ||
        (e = hipStreamSynchronize(s->stream)))
        return hip_fail(e, "read state");
    int flag = 0;
    std::memcpy(&flag, s->export_host + 6 * n, 4);
    std::memcpy(x_out, s->export_host, 12 * n);
    if (v_out) std::memcpy(v_out, s->export_host + 3 * n, 12 * n);
    if (flag & 2)
        return fail(CLOTH_ENAN, "a spring force exceeded the fixed-point accumulator's range "
                                "(8 N per component); use another kernel");
    if ((s->p.flags & CLOTH_F_CHECK_NAN) && (flag & 1))
        return fail(CLOTH_ENAN, "a non-finite value appeared in the state");
    return CLOTH_OK;
}

// First spring of each cloth of the handle, then the spring count.
std::vector<int> spring_segments(const cloth_sim* s) {
    std::vector<int> segs;
    for (const GroupInfo& g : s->groups) segs.push_back(g.spring_off);
    segs.push_back(s->n_springs);
    return segs;
}

// The grid stencil of the handle's cloths (build_stencil), on the device, when they have
// one; otherwise the grid kernel stays unavailable.
int build_stencil_device(cloth_sim* s) {
    std::vector<StencilCloth> sc;
    for (const GroupInfo& g : s->groups)
        sc.push_back(StencilCloth{g.nx, g.ny, g.node_off, g.slot_off, g.spring_off, g.n_springs});
    std::vector<int> code;
    std::vector<int4> tiles;
    if (!build_stencil(sc, s->ends, s->host.slot, s->dev.ld, &code, &tiles)) return CLOTH_OK;
    const size_t m = code.size(), ld = (size_t)s->dev.ld;
    const size_t G = s->groups.size();
    // bytes relative to the first entry of the slot's cloth
    const std::vector<int> bases = segment_bases(spring_segments(s), s->host.spring_entry);
    std::vector<int> slot_base(ld, 0);
    for (size_t g = 0; g < G; ++g)
        for (int q = s->group_off[g]; q < s->group_off[g + 1]; ++q) slot_base[q] = bases[g];
    std::vector<uint32_t> idx(m), idx8(m / 4, 0u);
    for (size_t q = 0; q < m; ++q) {
        idx[q] = code[q] >= 0 ? (uint32_t)s->host.spring_entry[code[q]] : kNoSpring;
        const size_t d = q / ld, p = q % ld;
        const uint32_t b =
            idx[q] == kNoSpring ? kNoSpring8 : ((idx[q] - (uint32_t)slot_base[p]) & 0xffu);
        idx8[(d / 4) * ld + p] |= b << (8 * (d % 4));
    }
    ClothDevice& d = s->dev;
    StreamFence fence{s->stream};
    hipError_t e;
    int *dc = nullptr, *dbase = nullptr;
    uint32_t *di = nullptr, *di8 = nullptr;
    int4* dt = nullptr;
    if ((e = s->arena.alloc(&dc, m)) || (e = s->arena.alloc(&di, m)) ||
        (e = s->arena.alloc(&di8, m / 4)) ||
        (G > 1 && (e = s->arena.alloc(&dt, tiles.size()))) ||
        (G > 1 && (e = s->arena.alloc(&dbase, G))) ||
        (dbase && (e = hipMemcpyAsync(dbase, bases.data(), 4 * G, hipMemcpyHostToDevice,
                                      s->stream))) ||
        (e = hipMemcpyAsync(dc, code.data(), 4 * m, hipMemcpyHostToDevice, s->stream)) ||
        (e = hipMemcpyAsync(di, idx.data(), 4 * m, hipMemcpyHostToDevice, s->stream)) ||
        (e = hipMemcpyAsync(di8, idx8.data(), m, hipMemcpyHostToDevice, s->stream)) ||
        (dt && (e = hipMemcpyAsync(dt, tiles.data(), tiles.size() * sizeof(int4),
                                   hipMemcpyHostToDevice, s->stream))) ||
        (e = hipStreamSynchronize(s->stream)))
        return hip_fail(e, "grid stencil");
    d.sten_code = dc;
    d.sten_idx = di;
    d.sten_idx8 = di8;
    d.tab_base = dbase;
    d.slot_cloth = G > 1 ? s->node_group_dev : nullptr;
    d.tiles = dt;
    d.n_tiles = (int)tiles.size();
    d.one_cloth = tiles.empty() ? int4{} : tiles[0];
    return CLOTH_OK;
}

int create_sim(const std::vector<ClothHostInput>& cloths, const cloth_params* p,
               hipStream_t stream, cloth_sim** out) {
    *out = nullptr;
    int st = validate_params(p);
    if (st != CLOTH_OK) return st;
    if (cloths.empty()) return fail(CLOTH_EINVAL, "no cloth");
    long long n_tot = 0, s_tot = 0;
    for (size_t g = 0; g < cloths.size(); ++g) {
        if ((st = validate_cloth(cloths[g])) != CLOTH_OK) {
            if (cloths.size() > 1) g_last_error = "cloth " + std::to_string(g) + ": " + g_last_error;
            return st;
        }
        n_tot += (long long)cloths[g].nx * cloths[g].ny;
        s_tot += cloths[g].n_springs;
    }
    if (n_tot > (1LL << 28) || s_tot > (1LL << 29)) return fail(CLOTH_EINVAL, "too many nodes or springs");
    cloth_sim* s = new (std::nothrow) cloth_sim();
    if (!s) return fail(CLOTH_ENOMEM, "host allocation failed");
    s->p = *p;
    s->stream = stream;
    s->n_nodes = (int)n_tot;
    s->n_springs = (int)s_tot;
    try {
        // merged arrays in caller numbering: cloth g's node i is node node_off_g + i
        std::vector<int> order;
        order.reserve((size_t)n_tot);
        s->x0.reserve(3 * (size_t)n_tot);
        std::vector<float> v0(3 * (size_t)n_tot, 0.0f);
        std::vector<float>& rest = s->rest;
        int node_off = 0;
        s->group_off.push_back(0);
        for (const auto& in : cloths) {
            GroupInfo g;
            g.nx = in.nx;
            g.ny = in.ny;
            g.n = in.nx * in.ny;
            g.node_off = node_off;
            g.slot_off = (int)order.size();
            g.n_springs = in.n_springs;
            g.spring_off = (int)s->k.size();
            for (int id : tile_order(in.nx, in.ny)) order.push_back(node_off + id);
            s->x0.insert(s->x0.end(), in.x0, in.x0 + 3 * (size_t)g.n);
            if (in.v0) std::copy(in.v0, in.v0 + 3 * (size_t)g.n, v0.begin() + 3 * (size_t)node_off);
            s->mass.insert(s->mass.end(), in.mass, in.mass + g.n);
            for (int i = 0; i < g.n; ++i) s->pinned.push_back(in.pinned && in.pinned[i] ? 1 : 0);
            for (int q = 0; q < 2 * in.n_springs; ++q) s->ends.push_back(in.ends[q] + node_off);
            rest.insert(rest.end(), in.rest, in.rest + in.n_springs);
            s->k.insert(s->k.end(), in.k, in.k + in.n_springs);
            s->c.insert(s->c.end(), in.c, in.c + in.n_springs);
            s->groups.push_back(g);
            node_off += g.n;
            s->group_off.push_back((int)order.size());
        }
        ClothHostInput merged{};
        merged.nx = (int)n_tot;
        merged.ny = 1;
        merged.x0 = s->x0.data();
        merged.v0 = v0.data();
        merged.mass = s->mass.data();
        merged.pinned = s->pinned.data();
        merged.n_springs = (int)s_tot;
        merged.ends = s->ends.data();
        merged.rest = rest.data();
        merged.k = s->k.data();
        merged.c = s->c.data();
        // parameter entries are distinct per cloth: each cloth's are one contiguous range
        const std::vector<int> segs = spring_segments(s);
        st = build_cloth_host(merged, &s->host, &order, &segs);
        for (size_t g = 0; g < cloths.size() && st == CLOTH_OK; ++g)
            stability_bounds(cloths[g], &s->groups[g].omega2, &s->groups[g].gamma);
    } catch (const std::bad_alloc&) {
        st = fail(CLOTH_ENOMEM, "host allocation failed");
    }
    if (st == CLOTH_OK) st = upload_cloth(s->host, s->arena, s->stream, &s->dev);
    if (st == CLOTH_OK) {
        s->surfs.resize(cloths.size());
        for (size_t g = 0; g < cloths.size() && st == CLOTH_OK; ++g) {
            st = build_surface(cloths[g], s->p, s->arena, s->stream, &s->surfs[g]);
            if (st != CLOTH_OK && cloths.size() > 1)
                g_last_error = "cloth " + std::to_string(g) + ": " + g_last_error;
            if (st == CLOTH_OK && s->surfs[g].view.n_tris > 0) s->any_collision = 1;
        }
        if (!s->any_collision) {
            // without collision the spring pass dominates, and for spring graphs off the grid
            // stencil the tile kernel's LDS gather is the faster default
            s->launch.kernel = CLOTH_KERNEL_TILE;
            s->launch.block_threads = 256;
        }
    }
    if (st == CLOTH_OK) {
        const size_t N = (size_t)n_tot, G = cloths.size();
        const size_t ld = (size_t)s->dev.ld;
        // host sources of the copies below; the fence waits for the copies before they go
        std::vector<SurfaceView> svs(G);
        std::vector<int> grp(G > 1 ? N : 0);
        StreamFence fence{s->stream};
        for (size_t g = 0; g < G; ++g) svs[g] = s->surfs[g].view;
        hipError_t e;
        if ((e = s->arena.alloc(&s->nan_flag, 1)) || (e = s->arena.alloc(&s->x_init, 3 * ld)) ||
            (e = s->arena.alloc(&s->v_init, 3 * ld)) || (e = s->arena.alloc(&s->slot_dev, N)) ||
            (e = s->arena.alloc(&s->svs_dev, G)) ||
            (e = hipMemsetAsync(s->nan_flag, 0, 4, s->stream)) ||
            (e = hipMemcpyAsync(s->svs_dev, svs.data(), G * sizeof(SurfaceView),
                                hipMemcpyHostToDevice, s->stream)) ||
            (e = hipMemcpyAsync(s->x_init, s->dev.x[0], 12 * ld, hipMemcpyDeviceToDevice, s->stream)) ||
            (e = hipMemcpyAsync(s->v_init, s->dev.v[0], 12 * ld, hipMemcpyDeviceToDevice, s->stream)) ||
            (e = hipMemcpyAsync(s->slot_dev, s->host.slot.data(), 4 * N, hipMemcpyHostToDevice,
                                s->stream)))
            st = hip_fail(e, "create");
        if (st == CLOTH_OK && G > 1) {
            for (size_t g = 0; g < G; ++g)
                for (int q = s->group_off[g]; q < s->group_off[g + 1]; ++q) grp[q] = (int)g;
            if ((e = s->arena.alloc(&s->node_group_dev, N)) ||
                (e = hipMemcpyAsync(s->node_group_dev, grp.data(), 4 * N, hipMemcpyHostToDevice,
                                    s->stream)))
                st = hip_fail(e, "create");
        }
        if (st == CLOTH_OK) st = build_stencil_device(s);
        if (st == CLOTH_OK && s->dev.sten_code) {
            // grid cloths: the stencil kernel is the faster default with a surface (16 against
            // 18 us per substep on the 316x316 workload) and without one (22 against 27 us for
            // the tile kernel on the 800x800 cloth).  Chunks of 16 tiles per XCD keep a tile's
            // halo rows in the L2 of the XCD that loaded them and still spread the tiles in
            // contact over every XCD: 19.6 -> 16.1 us per substep on the 800x800 cloth, 15.3
            // -> 14.7 us on the draped 316x316 cloth (hardware order, or one contiguous run
            // per XCD, which puts the contact region on one or two XCDs: 17.5 us)
            s->launch.kernel = CLOTH_KERNEL_GRID;
            s->launch.xcd_runs = 16;
            // a second wavefront per tile takes every other round of the narrow tests of the
            // nodes resting on the surface: 14.9 -> 13.8 us per substep on the draped 316x316
            // cloth, 7.0 -> 7.2 us in free fall; slower for the 512-cloth batch, whose
            // collision work is spread over many wavefronts (138 -> 187 us), so one there
            s->launch.block_threads = s->groups.size() == 1 && s->any_collision ? 128 : 64;
        }
        if (st == CLOTH_OK && (p->flags & CLOTH_F_NARROW_MT) && s->any_collision) {
            s->mt = true;
            if ((e = s->arena.alloc(&s->mt_pred, 6 * ld))) st = hip_fail(e, "create");
            if (st == CLOTH_OK) st = ensure_topology(s);
        }
        if (st == CLOTH_OK && (e = hipStreamSynchronize(s->stream))) st = hip_fail(e, "create");
    }
    if (st != CLOTH_OK) {
        delete s;
        return st;
    }
    s->host.release_state();
    *out = s;
    return CLOTH_OK;
}

int update_surface(cloth_sim* s, int group, const float* verts, int n_verts) {
    if (!verts) return fail(CLOTH_EINVAL, "verts is NULL");
    SurfaceDevice& sd = s->surfs[group];
    if (sd.view.n_tris == 0) return fail(CLOTH_EINVAL, "the cloth has no collision surface");
    if (n_verts != sd.n_verts)
        return fail(CLOTH_EINVAL, "n_verts must equal the surface's vertex count (" +
                                      std::to_string(sd.n_verts) + ")");
    const int st = rebuild_surface(&sd, verts, s->arena, s->stream);
    // a rebuild that failed after it started rewriting device arrays leaves that surface
    // inconsistent: the handle refuses to step until a rebuild of it succeeds
    s->surface_broken = false;
    for (const auto& other : s->surfs) s->surface_broken |= other.dirty;
    if (st != CLOTH_OK) return st;
    hipError_t e;
    if ((e = hipMemcpyAsync(s->svs_dev + group, &sd.view, sizeof(SurfaceView),
                            hipMemcpyHostToDevice, s->stream)) ||
        (e = hipStreamSynchronize(s->stream)))
        return hip_fail(e, "surface update");
    s->roll.ready = false;  // a rollout's contact sets were taken against the old surface
    return CLOTH_OK;
}

int set_external_force(cloth_sim* s, const float* f) {
    s->roll.ready = false;
    if (!f) {
        if (s->fext_on) s->drop_graphs();  // captured launches hold the force pointer
        s->fext_on = false;
        return CLOTH_OK;
    }
    const size_t N = (size_t)s->n_nodes, ld = (size_t)s->dev.ld;
    std::vector<float> soa(3 * ld, 0.0f);
    StreamFence fence{s->stream};
    for (size_t p = 0; p < N; ++p) {
        const size_t id = (size_t)s->host.order[p];
        for (int q = 0; q < 3; ++q) {
            const float v = f[3 * id + q];
            if (!std::isfinite(v)) return fail(CLOTH_EINVAL, "non-finite external force");
            soa[q * ld + p] = v;
        }
    }
    hipError_t e;
    if (!s->fext_dev && (e = s->arena.alloc(&s->fext_dev, 3 * ld))) return hip_fail(e, "hipMalloc force");
    if ((e = hipMemcpyAsync(s->fext_dev, soa.data(), 12 * ld, hipMemcpyHostToDevice, s->stream)) ||
        (e = hipStreamSynchronize(s->stream)))
        return hip_fail(e, "upload force");
    if (!s->fext_on) s->drop_graphs();
    s->fext_on = true;
    return CLOTH_OK;
}

int substeps_per_launch(const cloth_sim* s) {
    if (s->mt && s->any_collision) return 1;
    return s->launch.kernel == CLOTH_KERNEL_TILE ? s->launch.substeps_per_launch : 1;
}

int ensure_topology(cloth_sim* s) {
    hipError_t e;
    if (!s->order_dev) {
        const size_t G = s->groups.size();
        std::vector<int4> desc(G);
        StreamFence fence{s->stream};
        for (size_t g = 0; g < G; ++g)
            desc[g] = make_int4(s->groups[g].node_off, s->groups[g].nx, s->groups[g].ny, 0);
        int* order = nullptr;
        int4* gd = nullptr;
        if ((e = s->arena.alloc(&order, (size_t)s->n_nodes)) || (e = s->arena.alloc(&gd, G)) ||
            (e = hipMemcpyAsync(order, s->host.order.data(), 4 * (size_t)s->n_nodes,
                                hipMemcpyHostToDevice, s->stream)) ||
            (e = hipMemcpyAsync(gd, desc.data(), G * sizeof(int4), hipMemcpyHostToDevice,
                                s->stream)) ||
            (e = hipStreamSynchronize(s->stream)))
            return hip_fail(e, "normals set-up");
        s->order_dev = order;
        s->group_desc_dev = gd;
    }
    return CLOTH_OK;
}

int vertex_normals(cloth_sim* s, float* n_out) {
    if (!n_out) return fail(CLOTH_EINVAL, "n_out is NULL");
    int st = ensure_topology(s);
    if (st != CLOTH_OK) return st;
    hipError_t e;
    if ((e = launch_vertex_normals(s->n_nodes, s->dev.ld, s->dev.x[s->dev.cur], s->order_dev,
                                   s->slot_dev, s->node_group_dev, s->group_desc_dev, n_out,
                                   s->stream)))
        return hip_fail(e, "normals");
    return CLOTH_OK;
}

}  // namespace cloth

using namespace cloth;

extern "C" {

int cloth_create(int nx, int ny, const float* x0, const float* v0, const float* mass,
                 const unsigned char* pinned, int n_springs, const int* ends, const float* rest,
                 const float* k, const float* c, int n_verts, const float* verts, int n_tris,
                 const int* tris, const cloth_params* p, void* hip_stream, cloth_sim** out) {
    if (!out) return fail(CLOTH_EINVAL, "out is NULL");
    *out = nullptr;
    ClothHostInput in{nx, ny, x0, v0, mass, pinned, n_springs, ends, rest, k, c, n_verts, verts,
                      n_tris, tris};
    return create_sim({in}, p, (hipStream_t)hip_stream, out);
}

int cloth_step(cloth_sim* s, float dt, int n_substeps, int n_steps) {
    if (!s) return fail(CLOTH_EINVAL, "NULL handle");
    return step_sim(s, dt, n_substeps, n_steps);
}

int cloth_update_surface(cloth_sim* s, const float* verts, int n_verts) {
    if (!s) return fail(CLOTH_EINVAL, "NULL handle");
    if (s->groups.size() != 1) return fail(CLOTH_EINVAL, "use cloth_batch_update_surface for a batch");
    return update_surface(s, 0, verts, n_verts);
}

int cloth_set_external_force(cloth_sim* s, const float* f) {
    if (!s) return fail(CLOTH_EINVAL, "NULL handle");
    return set_external_force(s, f);
}

int cloth_vertex_normals(cloth_sim* s, float* n_out) {
    if (!s) return fail(CLOTH_EINVAL, "NULL handle");
    return vertex_normals(s, n_out);
}

int cloth_set_launch(cloth_sim* s, const cloth_launch* cfg) {
    if (!s || !cfg) return fail(CLOTH_EINVAL, "NULL argument");
    return set_launch(s, *cfg);
}

int cloth_get_launch(const cloth_sim* s, cloth_launch* cfg) {
    if (!s || !cfg) return fail(CLOTH_EINVAL, "NULL argument");
    *cfg = s->launch;
    return CLOTH_OK;
}

int cloth_read_state(const cloth_sim* s, float* x_out, float* v_out) {
    if (!s || !x_out) return fail(CLOTH_EINVAL, "NULL argument");
    if (s->groups.size() != 1) return fail(CLOTH_EINVAL, "use cloth_batch_read_state for a batch");
    return read_state_range(s, 0, x_out, v_out);
}

int cloth_write_state(cloth_sim* s, const float* x, const float* v) {
    if (!s || !x) return fail(CLOTH_EINVAL, "NULL argument");
    const int N = s->dev.n, ld = s->dev.ld;
    std::vector<float> xs(3 * (size_t)ld, 0.0f), vs(3 * (size_t)ld, 0.0f);
    StreamFence fence{s->stream};
    for (int p = 0; p < N; ++p) {
        const int id = s->host.order[p];
        for (int q = 0; q < 3; ++q) {
            const float xv = x[3 * (size_t)id + q];
            const float vv = v ? v[3 * (size_t)id + q] : 0.0f;
            if (!std::isfinite(xv) || !std::isfinite(vv)) return fail(CLOTH_EINVAL, "non-finite state");
            xs[(size_t)q * ld + p] = xv;
            vs[(size_t)q * ld + p] = vv;
        }
    }
    hipError_t e;
    if ((e = hipMemcpyAsync(s->dev.x[s->dev.cur], xs.data(), 12 * (size_t)ld, hipMemcpyHostToDevice,
                            s->stream)) ||
        (e = hipMemcpyAsync(s->dev.v[s->dev.cur], vs.data(), 12 * (size_t)ld, hipMemcpyHostToDevice,
                            s->stream)) ||
        (e = hipMemsetAsync(s->nan_flag, 0, 4, s->stream)) || (e = hipStreamSynchronize(s->stream)))
        return hip_fail(e, "write state");
    s->roll.ready = false;
    return CLOTH_OK;
}

int cloth_device_state(cloth_sim* s, float** x_soa, float** v_soa) {
    if (!s) return fail(CLOTH_EINVAL, "NULL handle");
    if (x_soa) *x_soa = s->dev.x[s->dev.cur];
    if (v_soa) *v_soa = s->dev.v[s->dev.cur];
    return CLOTH_OK;
}

int cloth_node_order(const cloth_sim* s, int* order) {
    if (!s || !order) return fail(CLOTH_EINVAL, "NULL argument");
    std::memcpy(order, s->host.order.data(), sizeof(int) * s->host.order.size());
    return CLOTH_OK;
}

int cloth_info(const cloth_sim* s, long long* out) {
    if (!s || !out) return fail(CLOTH_EINVAL, "NULL argument");
    const SurfaceDevice& sf = s->surfs[0];
    out[0] = s->dev.n;
    out[1] = s->n_springs;
    out[2] = sf.view.n_tris;
    out[3] = sf.n_cells;
    out[4] = sf.n_refs;
    for (int q = 0; q < 3; ++q) out[5 + q] = sf.view.n_tris ? sf.view.dim[q] : 0;
    return CLOTH_OK;
}

int cloth_destroy(cloth_sim* s) {
    if (!s) return CLOTH_OK;
    (void)hipStreamSynchronize(s->stream);
    delete s;
    return CLOTH_OK;
}

int cloth_debug_candidates(cloth_sim* s, int n_points, const float* points, int* pairs_out,
                           long long cap, long long* n_out) {
    if (!s || !n_out) return fail(CLOTH_EINVAL, "NULL argument");
    if (n_points < 0 || cap < 0) return fail(CLOTH_EINVAL, "negative size");
    if (n_points > 0 && !points) return fail(CLOTH_EINVAL, "points is NULL");
    if (cap > 0 && !pairs_out) return fail(CLOTH_EINVAL, "pairs_out is NULL");
    const SurfaceView& sv = s->surfs[0].view;
    if (sv.n_tris == 0) return fail(CLOTH_EINVAL, "collision is disabled for this handle");
    if (s->surface_broken) return fail(CLOTH_ESTATE, "a surface update failed; update it again first");
    *n_out = 0;
    if (n_points == 0) return CLOTH_OK;
    DeviceArena tmp;
    float* d_p;
    uint32_t *d_cnt, *d_off, *d_scan;
    hipError_t e;
    const size_t n = (size_t)n_points;
    if ((e = tmp.alloc(&d_p, 3 * n)) || (e = tmp.alloc(&d_cnt, n)) || (e = tmp.alloc(&d_off, n + 1)) ||
        (e = tmp.alloc(&d_scan, scan_tmp_words(n))))
        return hip_fail(e, "hipMalloc candidates");
    std::vector<float> soa(3 * n);
    for (size_t i = 0; i < n; ++i)
        for (int q = 0; q < 3; ++q) soa[q * n + i] = points[3 * i + q];
    uint32_t total = 0;
    StreamFence fence{s->stream};
    if ((e = hipMemcpyAsync(d_p, soa.data(), 12 * n, hipMemcpyHostToDevice, s->stream)) ||
        (e = launch_candidates_count(n_points, n_points, d_p, sv, s->launch.hit_slots, d_cnt,
                                     s->stream)) ||
        (e = scan_exclusive_u32(d_cnt, d_off, n, d_scan, s->stream)) ||
        (e = hipMemcpyAsync(&total, d_off + n, 4, hipMemcpyDeviceToHost, s->stream)) ||
        (e = hipStreamSynchronize(s->stream)))
        return hip_fail(e, "candidate count");
    *n_out = total;
    if (total == 0 || cap == 0) return CLOTH_OK;
    int* d_pairs;
    if ((e = tmp.alloc(&d_pairs, 2 * (size_t)total))) return hip_fail(e, "hipMalloc pairs");
    const size_t ncopy = (size_t)std::min<long long>(cap, total);
    if ((e = launch_candidates_write(n_points, n_points, d_p, sv, s->launch.hit_slots, d_off,
                                     d_pairs, s->stream)) ||
        (e = hipMemcpyAsync(pairs_out, d_pairs, 8 * ncopy, hipMemcpyDeviceToHost, s->stream)) ||
        (e = hipStreamSynchronize(s->stream)))
        return hip_fail(e, "candidate write");
    return CLOTH_OK;
}

int cloth_stability_bound(int n_nodes, const float* x0, const float* mass,
                          const unsigned char* pinned, int n_springs, const int* ends,
                          const float* k, const float* c, double* omega2, double* gamma) {
    if (!omega2 || !gamma) return fail(CLOTH_EINVAL, "NULL output");
    std::vector<float> rest((size_t)std::max(n_springs, 0), 1.0f);
    ClothHostInput in{n_nodes, 1, x0, nullptr, mass, pinned, n_springs, ends, rest.data(), k, c,
                      0, nullptr, 0, nullptr};
    if (int st = validate_cloth(in)) return st;
    stability_bounds(in, omega2, gamma);
    return CLOTH_OK;
}

const char* cloth_status_str(int status) {
    switch (status) {
        case CLOTH_OK: return "CLOTH_OK";
        case CLOTH_EINVAL: return "CLOTH_EINVAL: invalid argument";
        case CLOTH_ENOMEM: return "CLOTH_ENOMEM: out of memory or size limit";
        case CLOTH_EDEVICE: return "CLOTH_EDEVICE: HIP runtime or kernel failure";
        case CLOTH_EUNSTABLE: return "CLOTH_EUNSTABLE: substep exceeds the stability bound";
        case CLOTH_ESTATE: return "CLOTH_ESTATE: call out of order";
        case CLOTH_ENAN: return "CLOTH_ENAN: non-finite state";
        default: return "unknown cloth status";
    }
}

const char* cloth_last_error(void) { return g_last_error.c_str(); }

// --- batches (a5) ------------------------------------------------------------------
int cloth_batch_create(int n, const cloth_sim_desc* descs, const cloth_params* p,
                       void* hip_stream, cloth_batch** out) {
    if (!out) return fail(CLOTH_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || !descs) return fail(CLOTH_EINVAL, "need at least one cloth description");
    std::vector<ClothHostInput> cloths(n);
    for (int i = 0; i < n; ++i) {
        const cloth_sim_desc& d = descs[i];
        cloths[i] = ClothHostInput{d.nx, d.ny, d.x0, d.v0, d.mass, d.pinned, d.n_springs, d.ends,
                                   d.rest, d.k, d.c, d.n_verts, d.verts, d.n_tris, d.tris};
    }
    cloth_batch* b = new (std::nothrow) cloth_batch();
    if (!b) return fail(CLOTH_ENOMEM, "host allocation failed");
    const int st = create_sim(cloths, p, (hipStream_t)hip_stream, &b->sim);
    if (st != CLOTH_OK) {
        delete b;
        return st;
    }
    *out = b;
    return CLOTH_OK;
}

int cloth_batch_step(cloth_batch* b, float dt, int n_substeps, int n_steps) {
    if (!b) return fail(CLOTH_EINVAL, "NULL handle");
    return step_sim(b->sim, dt, n_substeps, n_steps);
}

int cloth_batch_read_state(const cloth_batch* b, int i, float* x_out, float* v_out) {
    if (!b || !x_out) return fail(CLOTH_EINVAL, "NULL argument");
    if (i < 0 || i >= (int)b->sim->groups.size()) return fail(CLOTH_EINVAL, "cloth index out of range");
    return read_state_range(b->sim, i, x_out, v_out);
}

int cloth_batch_update_surface(cloth_batch* b, int i, const float* verts, int n_verts) {
    if (!b) return fail(CLOTH_EINVAL, "NULL handle");
    if (i < 0 || i >= (int)b->sim->groups.size()) return fail(CLOTH_EINVAL, "cloth index out of range");
    return update_surface(b->sim, i, verts, n_verts);
}

int cloth_batch_set_external_force(cloth_batch* b, const float* f) {
    if (!b) return fail(CLOTH_EINVAL, "NULL handle");
    return set_external_force(b->sim, f);
}

int cloth_batch_vertex_normals(cloth_batch* b, float* n_out) {
    if (!b) return fail(CLOTH_EINVAL, "NULL handle");
    return vertex_normals(b->sim, n_out);
}

int cloth_batch_set_launch(cloth_batch* b, const cloth_launch* cfg) {
    if (!b || !cfg) return fail(CLOTH_EINVAL, "NULL argument");
    return set_launch(b->sim, *cfg);
}

int cloth_batch_get_launch(const cloth_batch* b, cloth_launch* cfg) {
    if (!b || !cfg) return fail(CLOTH_EINVAL, "NULL argument");
    *cfg = b->sim->launch;
    return CLOTH_OK;
}

int cloth_batch_autotune(cloth_batch* b, float dt, int n_substeps, int frames, cloth_launch* best) {
    if (!b) return fail(CLOTH_EINVAL, "NULL handle");
    return autotune_sim(b->sim, dt, n_substeps, frames, best);
}

int cloth_batch_info(const cloth_batch* b, long long* out) {
    if (!b || !out) return fail(CLOTH_EINVAL, "NULL argument");
    const cloth_sim* s = b->sim;
    long long tris = 0;
    for (const auto& sf : s->surfs) tris += sf.view.n_tris;
    out[0] = (long long)s->groups.size();
    out[1] = s->n_nodes;
    out[2] = s->n_springs;
    out[3] = tris;
    out[4] = s->plan.view.n_tiles;
    out[5] = s->plan.view.n_workgroups;
    return CLOTH_OK;
}

int cloth_batch_destroy(cloth_batch* b) {
    if (!b) return CLOTH_OK;
    delete b->sim;
    delete b;
    return CLOTH_OK;
}

}  // extern "C"
