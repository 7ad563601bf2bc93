// a5: batches of independent cloths of uneven sizes (cloth_batch_*).  A batch is one
// simulation handle holding every cloth: one node array, one tile plan whose tiles never
// cross two cloths, one surface grid per cloth, and one graph of launches for all of them.
#include <hip/hip_runtime.h>

#include <new>
#include <string>
#include <vector>

#include "sim.h"

using namespace cloth;

extern "C" {

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
