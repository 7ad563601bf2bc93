// a6: differentiable rollout (cloth_rollout_forward / cloth_rollout_backward) with
// checkpointed recomputation.  The forward pass records positions at the requested frames
// and (x, v) every ckpt_every frames; the backward pass walks the checkpoint segments from
// last to first, recomputes each segment's states from its checkpoint (bit-identical to the
// forward pass, so the contact sets are the same), and applies the substep adjoints in
// reverse.  Memory: one checkpoint per ckpt_every frames plus one segment of states.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "sim.h"

using namespace cloth;

namespace {

// Stiffness and damping from device arrays into every copy the handle keeps.
int set_spring_params(cloth_sim* s, const float* k_dev, const float* c_dev) {
    const size_t S = (size_t)s->n_springs;
    if (S == 0) return CLOTH_OK;
    hipError_t e;
    std::vector<float> k(S), c(S);
    StreamFence fence{s->stream};
    if ((e = hipMemcpyAsync(k.data(), k_dev, 4 * S, hipMemcpyDeviceToHost, s->stream)) ||
        (e = hipMemcpyAsync(c.data(), c_dev, 4 * S, hipMemcpyDeviceToHost, s->stream)) ||
        (e = hipStreamSynchronize(s->stream)))
        return hip_fail(e, "read spring parameters");
    for (size_t q = 0; q < S; ++q)
        if (!(k[q] >= 0.0f) || !std::isfinite(k[q]) || !(c[q] >= 0.0f) || !std::isfinite(c[q]))
            return fail(CLOTH_EINVAL, "spring " + std::to_string(q) + " needs finite k, c >= 0");
    s->k = k;
    s->c = c;
    // a new table of the distinct triples (one entry per spring at most: it fits in place)
    // and the records of the cloth and of the tile plan re-pointed at it
    const std::vector<int> segs = spring_segments(s);
    param_table(s->k.data(), s->c.data(), s->rest.data(), (int)S, &segs, &s->host.ptab,
                &s->host.spring_entry, &s->host.tab_span);
    int st = upload_param_table(s->host.ptab, s->host.spring_entry, s->host.tab_span,
                                segment_bases(segs, s->host.spring_entry), &s->dev,
                                s->host.inc_spring.size(), const_cast<uint2*>(s->plan.view.inc),
                                s->plan.inc_sid, s->plan.inc_count, s->stream);
    if (st != CLOTH_OK) return st;
    if (s->springs.ready &&
        (e = launch_set_params(S, s->springs.sid, k_dev, c_dev, s->springs.k, s->springs.c,
                               s->stream)))
        return hip_fail(e, "set spring-list parameters");
    refresh_stability(s);
    return CLOTH_OK;
}

StepParams step_params(const cloth_sim* s, float h) {
    StepParams sp;
    sp.h = h;
    for (int q = 0; q < 3; ++q) sp.g[q] = s->p.gravity[q];
    sp.restitution = s->p.restitution;
    sp.check_nan = 0;
    sp.nan_flag = s->nan_flag;
    sp.fext = s->fext_on ? s->fext_dev : nullptr;
    sp.fext_ld = s->dev.ld;
    return sp;
}

}  // namespace

extern "C" {

int cloth_rollout_forward(cloth_sim* s, const float* k_dev, const float* c_dev,
                          const float* v0_dev, float dt, int n_substeps, int n_steps,
                          int ckpt_every, const int* out_steps, int n_out, float* x_out_dev) {
    if (!s) return fail(CLOTH_EINVAL, "NULL handle");
    if (s->groups.size() != 1) return fail(CLOTH_EINVAL, "rollouts take a single-cloth handle");
    if (s->surface_broken) return fail(CLOTH_ESTATE, "a surface update failed; update it again first");
    if (s->mt) return fail(CLOTH_EINVAL, "rollouts use the point-triangle narrow phase");
    if (s->launch.kernel == CLOTH_KERNEL_SCATTER_F32 || s->launch.kernel == CLOTH_KERNEL_SCATTER_FIX)
        return fail(CLOTH_EINVAL, "rollouts recompute with the gather kernels: select the tile, "
                                  "direct or lanes kernel");
    if (s->n_springs > 0 && (!k_dev || !c_dev)) return fail(CLOTH_EINVAL, "k and c are required");
    if (!(dt > 0.0f) || !std::isfinite(dt) || n_substeps < 1 || n_steps < 0 || ckpt_every < 1)
        return fail(CLOTH_EINVAL, "need dt > 0, n_substeps >= 1, n_steps >= 0, ckpt_every >= 1");
    if (n_out < 0 || (n_out > 0 && (!out_steps || !x_out_dev)))
        return fail(CLOTH_EINVAL, "out_steps and x_out are required when n_out > 0");
    for (int j = 0; j < n_out; ++j)
        if (out_steps[j] < 0 || out_steps[j] > n_steps || (j && out_steps[j] < out_steps[j - 1]))
            return fail(CLOTH_EINVAL, "out_steps must be ascending frame counts in 0..n_steps");
    s->roll.ready = false;
    int st = set_spring_params(s, k_dev, c_dev);
    if (st != CLOTH_OK) return st;
    const float h = dt / (float)n_substeps;
    if (!(s->p.flags & CLOTH_F_NO_STABILITY_CHECK) &&
        unstable(s->groups[0].omega2, s->groups[0].gamma, h))
        return fail(CLOTH_EUNSTABLE, "substep exceeds the explicit stability bound");
    RolloutState& R = s->roll;
    const int N = s->dev.n;
    const size_t ld = (size_t)s->dev.ld, state = 6 * ld;
    R.h = h;
    R.n_sub = (long long)n_steps * n_substeps;
    R.ckpt = (long long)ckpt_every * n_substeps;
    R.n_ck = R.n_sub / R.ckpt + 1;
    R.out_sub.assign(n_out, 0);
    for (int j = 0; j < n_out; ++j) R.out_sub[j] = (long long)out_steps[j] * n_substeps;
    hipError_t e;
    if ((e = hipStreamSynchronize(s->stream))) return hip_fail(e, "synchronise");
    R.arena.release();
    R.seg = nullptr;
    R.pred = nullptr;
    R.adj = nullptr;
    R.kb = R.cb = nullptr;
    if ((e = R.arena.alloc(&R.ck, (size_t)R.n_ck * state)))
        return hip_fail(e, "hipMalloc checkpoints");
    // initial state: the handle's initial positions and the given velocities
    float* X = s->dev.x[s->dev.cur];
    float* V = s->dev.v[s->dev.cur];
    if ((e = hipMemcpyAsync(X, s->x_init, 12 * ld, hipMemcpyDeviceToDevice, s->stream)) ||
        (e = hipMemcpyAsync(V, s->v_init, 12 * ld, hipMemcpyDeviceToDevice, s->stream)) ||
        (v0_dev && (e = launch_import(N, (int)ld, s->slot_dev, v0_dev, V, 0, s->stream))) ||
        (e = hipMemsetAsync(s->nan_flag, 0, 4, s->stream)))
        return hip_fail(e, "rollout initial state");
    long long pos = 0;
    int j = 0;
    for (;;) {
        if (pos % R.ckpt == 0) {
            float* dst = R.ck + (size_t)(pos / R.ckpt) * state;
            if ((e = hipMemcpyAsync(dst, s->dev.x[s->dev.cur], 12 * ld, hipMemcpyDeviceToDevice,
                                    s->stream)) ||
                (e = hipMemcpyAsync(dst + 3 * ld, s->dev.v[s->dev.cur], 12 * ld,
                                    hipMemcpyDeviceToDevice, s->stream)))
                return hip_fail(e, "checkpoint");
        }
        while (j < n_out && R.out_sub[j] == pos) {
            if ((e = launch_export(N, (int)ld, s->slot_dev, s->dev.x[s->dev.cur],
                                   x_out_dev + (size_t)j * 3 * N, s->stream)))
                return hip_fail(e, "record output");
            ++j;
        }
        if (pos == R.n_sub) break;
        long long next = std::min(R.n_sub, (pos / R.ckpt + 1) * R.ckpt);
        if (j < n_out) next = std::min(next, R.out_sub[j]);
        if ((st = run_substeps(s, h, next - pos)) != CLOTH_OK) return st;
        pos = next;
    }
    R.ready = true;
    return CLOTH_OK;
}

int cloth_rollout_backward(cloth_sim* s, const float* gx_out_dev, float* gk_dev, float* gc_dev,
                           float* gv0_dev) {
    if (!s) return fail(CLOTH_EINVAL, "NULL handle");
    RolloutState& R = s->roll;
    if (!R.ready) return fail(CLOTH_ESTATE, "cloth_rollout_backward needs a preceding forward pass");
    if (!R.out_sub.empty() && !gx_out_dev) return fail(CLOTH_EINVAL, "gx_out is required");
    const int N = s->dev.n, n_out = (int)R.out_sub.size();
    const size_t ld = (size_t)s->dev.ld, S = (size_t)s->n_springs, state = 6 * ld;
    hipError_t e;
    if (!R.seg) {
        if ((e = R.arena.alloc(&R.seg, (size_t)(R.ckpt + 1) * state)) ||
            (e = R.arena.alloc(&R.pred, (size_t)R.ckpt * 3 * ld)) ||
            (e = R.arena.alloc(&R.adj, 7 * 3 * ld)) || (e = R.arena.alloc(&R.kb, S + 1)) ||
            (e = R.arena.alloc(&R.cb, S + 1)))
            return hip_fail(e, "hipMalloc adjoint buffers");
    }
    int st = ensure_topology(s);  // the slot -> node order, for outputs added in a fused launch
    if (st != CLOTH_OK) return st;
    float* xb = R.adj;
    float* vb = R.adj + 3 * ld;
    float* fb = R.adj + 6 * ld;
    float* fb2 = R.adj + 9 * ld;
    float* xbp = R.adj + 15 * ld;
    float* vbp = R.adj + 18 * ld;
    if ((e = hipMemsetAsync(xb, 0, 4 * 6 * ld, s->stream)) ||
        (e = hipMemsetAsync(R.kb, 0, 8 * (S + 1), s->stream)) ||
        (e = hipMemsetAsync(R.cb, 0, 8 * (S + 1), s->stream)))
        return hip_fail(e, "clear adjoints");
    const ClothView cv = s->dev.view();
    const StepParams sp = step_params(s, R.h);
    int j = n_out - 1;
    auto add_outputs = [&](long long at) -> hipError_t {
        while (j >= 0 && R.out_sub[j] == at) {
            hipError_t r = launch_import(N, (int)ld, s->slot_dev, gx_out_dev + (size_t)j * 3 * N,
                                         xb, 1, s->stream);
            if (r != hipSuccess) return r;
            --j;
        }
        return hipSuccess;
    };
    if ((e = add_outputs(R.n_sub))) return hip_fail(e, "seed adjoint");
    for (long long seg = (R.n_sub - 1) / R.ckpt; seg >= 0 && R.n_sub > 0; --seg) {
        const long long base = seg * R.ckpt, top = std::min(base + R.ckpt, R.n_sub);
        if ((e = hipMemcpyAsync(R.seg, R.ck + (size_t)seg * state, 4 * state,
                                hipMemcpyDeviceToDevice, s->stream)))
            return hip_fail(e, "restore checkpoint");
        // the segment's states and every substep's prediction (substep r of the segment
        // stores it at pred[r - 1]); the listed collision query, as the forward pass (any
        // launch gives the same bits)
        const bool collide = s->surfs[0].view.n_tris > 0;
        for (long long r = 1; r <= top - base; ++r) {
            const float* xs = R.seg + (size_t)(r - 1) * state;
            float* xd = R.seg + (size_t)r * state;
            float* pr = R.pred + (size_t)(r - 1) * 3 * ld;
            e = s->dev.sten_code
                    ? launch_grid_substep(cv, s->dev.grid_view(), collide, sp, xs, xs + 3 * ld, xd,
                                          xd + 3 * ld, s->stream, s->svs_dev, 0,
                                          s->launch.hit_slots, s->launch.xcd_runs,
                                          s->launch.kernel == CLOTH_KERNEL_GRID
                                              ? s->launch.block_threads / 64
                                              : 1,
                                          pr)
                    : launch_substep(cv, collide, sp, xs, xs + 3 * ld, xd, xd + 3 * ld, 256,
                                     s->stream, s->svs_dev, nullptr, s->launch.hit_slots, 0, 0,
                                     nullptr, 0, pr);
            if (e) return hip_fail(e, "recompute segment");
        }
        // (xb, vb) hold the adjoint of the state after substep top.  The node pass of
        // substep t needs the state before it, s[t - 1]; the spring pass of substep t and the
        // node pass of substep t - 1 run as one launch while both states are in the segment.
        const SurfaceView& sv0 = s->surfs[0].view;
        const int slots = s->launch.hit_slots;
        auto state_at = [&](long long t) { return R.seg + (size_t)(t - base) * state; };
        auto pred_of = [&](long long t) { return R.pred + (size_t)(t - 1 - base) * 3 * ld; };
        if ((e = launch_adj_node(cv, sv0, sp, state_at(top - 1), state_at(top - 1) + 3 * ld, xb, vb,
                                 fb, xbp, vbp, slots, pred_of(top), s->stream)))
            return hip_fail(e, "adjoint substep");
        for (long long t = top; t > base; --t) {
            const float* xa = state_at(t - 1);
            int outs = 0;  // outputs recorded at the state between substeps t - 1 and t
            while (j - outs >= 0 && R.out_sub[j - outs] == t - 1) ++outs;
            if (t - 1 > base && outs <= 1) {
                const float* xbs = state_at(t - 2);
                const float* gout = outs ? gx_out_dev + (size_t)j * 3 * N : nullptr;
                if ((e = launch_adj_fused(cv, sv0, sp, xa, xa + 3 * ld, xbs, xbs + 3 * ld,
                                          pred_of(t - 1), fb, fb2, xbp, vbp, xb, vb, R.kb, R.cb,
                                          gout, s->order_dev, slots, s->stream)))
                    return hip_fail(e, "adjoint substep");
                j -= outs;
                std::swap(fb, fb2);
            } else {
                if ((e = launch_adj_springs(cv, xa, xa + 3 * ld, fb, xbp, vbp, xb, vb, R.kb, R.cb,
                                            s->stream)) ||
                    (e = add_outputs(t - 1)))
                    return hip_fail(e, "adjoint substep");
                if (t - 1 > base &&
                    (e = launch_adj_node(cv, sv0, sp, state_at(t - 2), state_at(t - 2) + 3 * ld, xb,
                                         vb, fb, xbp, vbp, slots, pred_of(t - 1), s->stream)))
                    return hip_fail(e, "adjoint substep");
            }
        }
    }
    if ((gv0_dev && (e = launch_export(N, (int)ld, s->slot_dev, vb, gv0_dev, s->stream))) ||
        (gk_dev && (e = launch_d2f(S, R.kb, gk_dev, s->stream))) ||
        (gc_dev && (e = launch_d2f(S, R.cb, gc_dev, s->stream))))
        return hip_fail(e, "write gradients");
    return CLOTH_OK;
}

int cloth_debug_contacts(cloth_sim* s, float h, int* counts, int* ids, int cap) {
    if (!s || !counts) return fail(CLOTH_EINVAL, "NULL argument");
    if (s->groups.size() != 1) return fail(CLOTH_EINVAL, "single-cloth handles only");
    if (s->surface_broken) return fail(CLOTH_ESTATE, "a surface update failed; update it again first");
    if (!(h > 0.0f) || !std::isfinite(h) || cap < 0 || (cap > 0 && !ids))
        return fail(CLOTH_EINVAL, "need h > 0 and ids when cap > 0");
    const int N = s->dev.n;
    DeviceArena tmp;
    int *d_cnt, *d_ids;
    hipError_t e;
    if ((e = tmp.alloc(&d_cnt, (size_t)N)) || (e = tmp.alloc(&d_ids, (size_t)N * cap + 1)))
        return hip_fail(e, "hipMalloc contacts");
    std::vector<int> cnt(N), id((size_t)N * cap + 1);
    StreamFence fence{s->stream};
    const hipError_t le =
        s->mt ? launch_mt_debug_contacts(s->dev.view(), step_params(s, h),
                                         MtTopology{s->order_dev, s->slot_dev, nullptr,
                                                    s->group_desc_dev},
                                         s->svs_dev, s->dev.x[s->dev.cur], s->dev.v[s->dev.cur],
                                         s->mt_pred, d_cnt, d_ids, cap, s->stream)
              : launch_debug_contacts(s->dev.view(), s->surfs[0].view, step_params(s, h),
                                      s->dev.x[s->dev.cur], s->dev.v[s->dev.cur], d_cnt, d_ids,
                                      cap, s->launch.hit_slots, s->stream);
    if ((e = le) ||
        (e = hipMemcpyAsync(cnt.data(), d_cnt, 4 * (size_t)N, hipMemcpyDeviceToHost, s->stream)) ||
        (cap > 0 && (e = hipMemcpyAsync(id.data(), d_ids, 4 * (size_t)N * cap,
                                        hipMemcpyDeviceToHost, s->stream))) ||
        (e = hipStreamSynchronize(s->stream)))
        return hip_fail(e, "debug contacts");
    for (int p = 0; p < N; ++p) {
        const int node = s->host.order[p];
        counts[node] = cnt[p];
        // the triangle-triangle search lists contacts in its candidate order
        if (s->mt) std::sort(id.begin() + (size_t)p * cap, id.begin() + (size_t)p * cap + std::min(cnt[p], cap));
        for (int r = 0; r < cap; ++r) ids[(size_t)node * cap + r] = id[(size_t)p * cap + r];
    }
    return CLOTH_OK;
}

int cloth_debug_query_volume(cloth_sim* s, float h, long long* out) {
    if (!s || !out) return fail(CLOTH_EINVAL, "NULL argument");
    if (s->groups.size() != 1) return fail(CLOTH_EINVAL, "single-cloth handles only");
    if (s->mt) return fail(CLOTH_EINVAL, "the proximity query only (not CLOTH_F_NARROW_MT)");
    if (s->surface_broken) return fail(CLOTH_ESTATE, "a surface update failed; update it again first");
    if (!(h > 0.0f) || !std::isfinite(h)) return fail(CLOTH_EINVAL, "need h > 0");
    for (int q = 0; q < 6; ++q) out[q] = 0;
    const SurfaceView& sv = s->surfs[0].view;
    if (sv.n_tris == 0) return CLOTH_OK;
    const size_t C = (size_t)sv.dim[0] * sv.dim[1] * sv.dim[2];
    const size_t cw = (C + 31) / 32, tw = ((size_t)sv.n_tris + 31) / 32;
    DeviceArena tmp;
    uint32_t *d_cb, *d_tb;
    unsigned long long* d_tot;
    hipError_t e;
    if ((e = tmp.alloc(&d_cb, cw)) || (e = tmp.alloc(&d_tb, tw)) || (e = tmp.alloc(&d_tot, 3)))
        return hip_fail(e, "hipMalloc query volume");
    std::vector<uint32_t> cb(cw), tb(tw), start(C + 1);
    unsigned long long tot[3] = {0, 0, 0};
    StreamFence fence{s->stream};
    if ((e = hipMemsetAsync(d_cb, 0, 4 * cw, s->stream)) ||
        (e = hipMemsetAsync(d_tb, 0, 4 * tw, s->stream)) ||
        (e = hipMemsetAsync(d_tot, 0, 24, s->stream)) ||
        (e = launch_debug_volume(s->dev.view(), sv, step_params(s, h), s->dev.x[s->dev.cur],
                                 s->dev.v[s->dev.cur], s->launch.hit_slots, d_cb, d_tb, d_tot,
                                 s->stream)) ||
        (e = hipMemcpyAsync(cb.data(), d_cb, 4 * cw, hipMemcpyDeviceToHost, s->stream)) ||
        (e = hipMemcpyAsync(tb.data(), d_tb, 4 * tw, hipMemcpyDeviceToHost, s->stream)) ||
        (e = hipMemcpyAsync(start.data(), sv.cell_start, 4 * (C + 1), hipMemcpyDeviceToHost,
                            s->stream)) ||
        (e = hipMemcpyAsync(tot, d_tot, 24, hipMemcpyDeviceToHost, s->stream)) ||
        (e = hipStreamSynchronize(s->stream)))
        return hip_fail(e, "query volume");
    long long cells = 0, refs = 0, tris = 0;
    for (size_t w = 0; w < cw; ++w)
        for (uint32_t m = cb[w]; m; m &= m - 1) {
            const size_t c = 32 * w + (size_t)__builtin_ctz(m);
            ++cells;
            refs += (long long)(start[c + 1] - start[c]);
        }
    for (size_t w = 0; w < tw; ++w) tris += __builtin_popcount(tb[w]);
    out[0] = cells;
    out[1] = refs;
    out[2] = tris;
    out[3] = (long long)tot[0];
    out[4] = (long long)tot[1];
    out[5] = (long long)tot[2];
    return CLOTH_OK;
}

}  // extern "C"
