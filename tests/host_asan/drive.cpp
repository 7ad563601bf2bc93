// Drives every host path of the C ABI (include/cloth.h) once, against the stand-in runtime of
// hip_stub.cpp: plain, batched and triangle-triangle handles, launch configurations and tile
// schedules, autotuning, state access, surface updates, external forces, normals, debug
// queries, rollouts and error paths.  Built with AddressSanitizer and
// UndefinedBehaviorSanitizer; prints "host paths ok" and exits 0 when nothing was reported.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/cloth.h"

namespace {

int g_fail = 0;

void expect(int got, int want, const char* what) {
    if (got != want) {
        std::fprintf(stderr, "%s: status %d (want %d): %s\n", what, got, want, cloth_last_error());
        g_fail = 1;
    }
}

// An n x n cloth of spacing 0.01 at height y over a regular octahedron of radius 0.2 (or no
// surface): structural, shear and bend springs, k = 500 / 200 / 50, c = 0.05, 1 g per node.
struct Cloth {
    int n = 0;
    std::vector<float> x0, v0, mass, rest, k, c, verts;
    std::vector<int> ends, tris;
    std::vector<unsigned char> pinned;
};

Cloth make_cloth(int n, bool surface, bool pin_corners) {
    Cloth cl;
    cl.n = n;
    const float s = 0.01f;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            cl.x0.insert(cl.x0.end(), {(j - 0.5f * (n - 1)) * s, 0.3f, (i - 0.5f * (n - 1)) * s});
            cl.v0.insert(cl.v0.end(), {0.0f, 0.0f, 0.0f});
            cl.mass.push_back(1e-3f);
            cl.pinned.push_back(pin_corners && i == 0 && (j == 0 || j == n - 1));
        }
    auto spring = [&](int i0, int j0, int i1, int j1, float kk, float len) {
        if (i1 < 0 || j1 < 0 || i1 >= n || j1 >= n) return;
        cl.ends.push_back(i0 * n + j0);
        cl.ends.push_back(i1 * n + j1);
        cl.rest.push_back(len);
        cl.k.push_back(kk);
        cl.c.push_back(0.05f);
    };
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            spring(i, j, i, j + 1, 500.0f, s);
            spring(i, j, i + 1, j, 500.0f, s);
            spring(i, j, i + 1, j + 1, 200.0f, s * std::sqrt(2.0f));
            spring(i, j, i + 1, j - 1, 200.0f, s * std::sqrt(2.0f));
            spring(i, j, i, j + 2, 50.0f, 2 * s);
            spring(i, j, i + 2, j, 50.0f, 2 * s);
        }
    if (surface) {
        const float r = 0.2f;
        cl.verts = {r, 0, 0, -r, 0, 0, 0, r, 0, 0, -r, 0, 0, 0, r, 0, 0, -r};
        cl.tris = {0, 2, 4, 2, 1, 4, 1, 3, 4, 3, 0, 4, 2, 0, 5, 1, 2, 5, 3, 1, 5, 0, 3, 5};
    }
    return cl;
}

cloth_params params(unsigned flags) {
    cloth_params p{};
    p.gravity[1] = -9.81f;
    p.thickness = 0.005f;
    p.cell_size = 0.0f;
    p.restitution = 0.5f;
    p.flags = flags;
    return p;
}

int create(const Cloth& cl, unsigned flags, cloth_sim** out) {
    const cloth_params p = params(flags);
    return cloth_create(cl.n, cl.n, cl.x0.data(), cl.v0.data(), cl.mass.data(), cl.pinned.data(),
                        (int)cl.k.size(), cl.ends.data(), cl.rest.data(), cl.k.data(),
                        cl.c.data(), (int)cl.verts.size() / 3, cl.verts.data(),
                        (int)cl.tris.size() / 3, cl.tris.data(), &p, nullptr, out);
}

cloth_launch tile_launch(int tile, int K, int sched, int wg) {
    return cloth_launch{CLOTH_KERNEL_TILE, tile, K, 256, 1, sched, wg, 32, 0, 0};
}

void plain_paths() {
    const float dt = 1.0f / 600.0f;
    Cloth cl = make_cloth(40, true, false);
    cloth_sim* s = nullptr;
    expect(create(cl, 0, &s), CLOTH_OK, "create");
    if (!s) return;
    const int N = cl.n * cl.n;
    expect(cloth_step(s, dt, 4, 10), CLOTH_OK, "step (graph replay)");
    expect(cloth_step(s, dt, 1, 1), CLOTH_EUNSTABLE, "step (too long a substep)");
    std::vector<float> x(3 * N), v(3 * N);
    expect(cloth_read_state(s, x.data(), v.data()), CLOTH_OK, "read state");
    expect(cloth_write_state(s, cl.x0.data(), nullptr), CLOTH_OK, "write state");
    const cloth_launch cfgs[] = {
        tile_launch(64, 1, CLOTH_SCHED_GRID, 0), tile_launch(256, 2, CLOTH_SCHED_LPT, 7),
        tile_launch(128, 4, CLOTH_SCHED_RR, 5), {CLOTH_KERNEL_DIRECT, 256, 1, 128, 1, 0, 0, 16, 2, 48},
        {CLOTH_KERNEL_SCATTER_FIX, 256, 1, 256, 0, 0, 0, 0, 0, 0},
        {CLOTH_KERNEL_SCATTER_F32, 256, 1, 64, 1, 0, 0, 8, 1, 0},
        {CLOTH_KERNEL_LANES4, 256, 1, 64, 1, 0, 0, 8, 0, 0},
        {CLOTH_KERNEL_LANES2, 256, 1, 256, 0, 0, 0, 0, 3, 0},
        {CLOTH_KERNEL_GRID, 256, 1, 64, 1, 0, 0, 32, 2, 0}};
    for (const cloth_launch& c : cfgs) {
        expect(cloth_set_launch(s, &c), CLOTH_OK, "set launch");
        expect(cloth_step(s, dt, 4, 9), CLOTH_OK, "step");
    }
    cloth_launch bad = tile_launch(96, 1, 0, 0);
    expect(cloth_set_launch(s, &bad), CLOTH_EINVAL, "set launch (bad tile)");
    cloth_launch best{};
    expect(cloth_autotune(s, dt, 4, 2, &best), CLOTH_OK, "autotune");
    std::vector<int> pairs(2 * 64);
    long long n_pairs = 0;
    expect(cloth_debug_candidates(s, N, x.data(), pairs.data(), 64, &n_pairs), CLOTH_OK,
           "debug candidates");
    std::vector<int> counts(N), ids(4 * N);
    expect(cloth_debug_contacts(s, dt / 4, counts.data(), ids.data(), 4), CLOTH_OK,
           "debug contacts");
    long long volume[6];
    expect(cloth_debug_query_volume(s, dt / 4, volume), CLOTH_OK, "query volume");
    expect(cloth_debug_query_volume(s, dt / 4, nullptr), CLOTH_EINVAL, "query volume (NULL)");
    std::vector<float> f(3 * N, 0.001f);
    expect(cloth_set_external_force(s, f.data()), CLOTH_OK, "external force");
    expect(cloth_step(s, dt, 4, 9), CLOTH_OK, "step (forced)");
    expect(cloth_set_external_force(s, nullptr), CLOTH_OK, "external force off");
    std::vector<float> moved(cl.verts);
    for (size_t q = 0; q < moved.size(); q += 3) moved[q] += 0.01f;
    expect(cloth_update_surface(s, moved.data(), (int)moved.size() / 3), CLOTH_OK,
           "update surface");
    moved[4] = NAN;
    expect(cloth_update_surface(s, moved.data(), (int)moved.size() / 3), CLOTH_EINVAL,
           "update surface (non-finite)");
    float* normals = nullptr;
    (void)hipMalloc((void**)&normals, 12 * (size_t)N);
    expect(cloth_vertex_normals(s, normals), CLOTH_OK, "normals");
    // a rollout with device arrays
    const int S = (int)cl.k.size();
    float *k_dev, *c_dev, *v0_dev, *xo_dev, *gk, *gc, *gv0;
    (void)hipMalloc((void**)&k_dev, 4 * (size_t)S);
    (void)hipMalloc((void**)&c_dev, 4 * (size_t)S);
    (void)hipMalloc((void**)&v0_dev, 12 * (size_t)N);
    (void)hipMalloc((void**)&xo_dev, 2 * 12 * (size_t)N);
    (void)hipMalloc((void**)&gk, 4 * (size_t)S);
    (void)hipMalloc((void**)&gc, 4 * (size_t)S);
    (void)hipMalloc((void**)&gv0, 12 * (size_t)N);
    (void)hipMemcpyAsync(k_dev, cl.k.data(), 4 * (size_t)S, hipMemcpyHostToDevice, nullptr);
    (void)hipMemcpyAsync(c_dev, cl.c.data(), 4 * (size_t)S, hipMemcpyHostToDevice, nullptr);
    (void)hipStreamSynchronize(nullptr);
    const cloth_launch direct{CLOTH_KERNEL_DIRECT, 256, 1, 64, 1, 0, 0, 32, 0, 0};
    expect(cloth_set_launch(s, &direct), CLOTH_OK, "set launch (direct)");
    expect(cloth_rollout_backward(s, xo_dev, gk, gc, gv0), CLOTH_ESTATE, "backward first");
    const int outs[2] = {5, 12};
    expect(cloth_rollout_forward(s, k_dev, c_dev, v0_dev, dt, 4, 12, 5, outs, 2, xo_dev),
           CLOTH_OK, "rollout forward");
    expect(cloth_rollout_backward(s, xo_dev, gk, gc, gv0), CLOTH_OK, "rollout backward");
    expect(cloth_rollout_backward(s, xo_dev, gk, gc, gv0), CLOTH_OK, "rollout backward again");
    for (float* p : {k_dev, c_dev, v0_dev, xo_dev, gk, gc, gv0, normals}) (void)hipFree(p);
    expect(cloth_destroy(s), CLOTH_OK, "destroy");
    // the triangle-triangle narrow phase
    expect(create(cl, CLOTH_F_NARROW_MT, &s), CLOTH_OK, "create (MT)");
    if (s) {
        expect(cloth_step(s, dt, 4, 9), CLOTH_OK, "step (MT)");
        expect(cloth_debug_contacts(s, dt / 4, counts.data(), ids.data(), 4), CLOTH_OK,
               "debug contacts (MT)");
        expect(cloth_destroy(s), CLOTH_OK, "destroy (MT)");
    }
    // invalid inputs
    Cloth broken = make_cloth(8, true, true);
    broken.ends[7] = broken.ends[6];
    expect(create(broken, 0, &s), CLOTH_EINVAL, "create (self spring)");
    Cloth hanging = make_cloth(24, false, true);
    expect(create(hanging, 0, &s), CLOTH_OK, "create (no surface)");
    if (s) {
        expect(cloth_step(s, 1.0f / 1200.0f, 2, 17), CLOTH_OK, "step (tile default)");
        expect(cloth_destroy(s), CLOTH_OK, "destroy");
    }
}

void batch_paths() {
    const float dt = 1.0f / 600.0f;
    const int n = 48;
    std::vector<Cloth> cl;
    unsigned r = 12345u;
    for (int i = 0; i < n; ++i) {
        r = r * 1103515245u + 12345u;
        cl.push_back(make_cloth(16 + (int)((r >> 16) % 49), true, false));
    }
    std::vector<cloth_sim_desc> d(n);
    long long nodes = 0;
    for (int i = 0; i < n; ++i) {
        const Cloth& c = cl[i];
        d[i] = cloth_sim_desc{c.n, c.n, c.x0.data(), c.v0.data(), c.mass.data(), c.pinned.data(),
                              (int)c.k.size(), c.ends.data(), c.rest.data(), c.k.data(),
                              c.c.data(), (int)c.verts.size() / 3, c.verts.data(),
                              (int)c.tris.size() / 3, c.tris.data()};
        nodes += (long long)c.n * c.n;
    }
    const cloth_params p = params(0);
    cloth_batch* b = nullptr;
    expect(cloth_batch_create(n, d.data(), &p, nullptr, &b), CLOTH_OK, "batch create");
    if (!b) return;
    expect(cloth_batch_step(b, dt, 4, 10), CLOTH_OK, "batch step");
    const cloth_launch cfgs[] = {tile_launch(256, 2, CLOTH_SCHED_LPT, 512),
                                 tile_launch(128, 1, CLOTH_SCHED_RR, 9),
                                 tile_launch(64, 4, CLOTH_SCHED_GRID, 0)};
    for (const cloth_launch& c : cfgs) {
        expect(cloth_batch_set_launch(b, &c), CLOTH_OK, "batch set launch");
        expect(cloth_batch_step(b, dt, 4, 9), CLOTH_OK, "batch step");
    }
    cloth_launch best{};
    expect(cloth_batch_autotune(b, dt, 4, 2, &best), CLOTH_OK, "batch autotune");
    long long info[6];
    expect(cloth_batch_info(b, info), CLOTH_OK, "batch info");
    for (int i : {0, n / 2, n - 1}) {
        std::vector<float> x(3 * (size_t)cl[i].n * cl[i].n);
        expect(cloth_batch_read_state(b, i, x.data(), nullptr), CLOTH_OK, "batch read state");
        expect(cloth_batch_update_surface(b, i, cl[i].verts.data(), (int)cl[i].verts.size() / 3),
               CLOTH_OK, "batch update surface");
    }
    std::vector<float> f(3 * (size_t)nodes, 0.0f);
    expect(cloth_batch_set_external_force(b, f.data()), CLOTH_OK, "batch external force");
    float* normals = nullptr;
    (void)hipMalloc((void**)&normals, 12 * (size_t)nodes);
    expect(cloth_batch_vertex_normals(b, normals), CLOTH_OK, "batch normals");
    (void)hipFree(normals);
    expect(cloth_batch_destroy(b), CLOTH_OK, "batch destroy");
    // a batch with one invalid cloth
    std::vector<float> bad_mass(cl[5].mass);
    bad_mass[3] = 0.0f;
    d[5].mass = bad_mass.data();
    expect(cloth_batch_create(n, d.data(), &p, nullptr, &b), CLOTH_EINVAL, "batch create (bad)");
}

}  // namespace

int main() {
    plain_paths();
    batch_paths();
    if (g_fail) return 1;
    std::printf("host paths ok\n");
    return 0;
}
