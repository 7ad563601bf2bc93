// Host side of the C ABI (include/cloth.h): input validation, the internal node order, the
// sliced CSR incidence build, the stability bound, the surface grid build, and stepping.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/cloth.h"
#include "cloth_internal.h"
#include "host_common.h"

using namespace cloth;

// ------------------------------------------------------------------ error plumbing

namespace cloth {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(CLOTH_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

DeviceArena::~DeviceArena() { release(); }

void DeviceArena::release() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
}

hipError_t DeviceArena::alloc_bytes(void** p, size_t bytes) {
    *p = nullptr;
    hipError_t e = hipMalloc(p, bytes ? bytes : 16);
    if (e == hipSuccess) ptrs.push_back(*p);
    return e;
}

void DeviceArena::free_one(void* p) {
    if (!p) return;
    auto it = std::find(ptrs.begin(), ptrs.end(), p);
    if (it != ptrs.end()) {
        (void)hipFree(p);
        ptrs.erase(it);
    }
}

// Internal node order: the nx-by-ny grid cut into 8x8 tiles, tiles in row-major order,
// nodes row-major within a tile, so a wavefront of 64 consecutive slots covers a compact
// patch of cloth.
std::vector<int> tile_order(int nx, int ny) {
    const int T = 8;
    std::vector<int> order;
    order.reserve((size_t)nx * ny);
    for (int ty = 0; ty < ny; ty += T)
        for (int tx = 0; tx < nx; tx += T)
            for (int i = ty; i < std::min(ny, ty + T); ++i)
                for (int j = tx; j < std::min(nx, tx + T); ++j) order.push_back(i * nx + j);
    return order;
}

int validate_cloth(const ClothHostInput& in) {
    if (in.nx <= 0 || in.ny <= 0) return fail(CLOTH_EINVAL, "nx and ny must be positive");
    const long long N = (long long)in.nx * in.ny;
    if (N > (1LL << 28)) return fail(CLOTH_EINVAL, "too many nodes");
    if (!in.x0 || !in.mass) return fail(CLOTH_EINVAL, "x0 and mass are required");
    if (in.n_springs < 0) return fail(CLOTH_EINVAL, "n_springs < 0");
    if (in.n_springs > 0 && (!in.ends || !in.rest || !in.k || !in.c))
        return fail(CLOTH_EINVAL, "ends, rest, k and c are required when n_springs > 0");
    for (long long i = 0; i < 3 * N; ++i) {
        if (!std::isfinite(in.x0[i])) return fail(CLOTH_EINVAL, "non-finite x0");
        if (in.v0 && !std::isfinite(in.v0[i])) return fail(CLOTH_EINVAL, "non-finite v0");
    }
    for (long long i = 0; i < N; ++i) {
        const bool pin = in.pinned && in.pinned[i];
        if (!pin && !(in.mass[i] > 0.0f && std::isfinite(in.mass[i])))
            return fail(CLOTH_EINVAL, "mass must be positive and finite on unpinned node " +
                                          std::to_string(i));
    }
    for (int s = 0; s < in.n_springs; ++s) {
        const int a = in.ends[2 * s], b = in.ends[2 * s + 1];
        if (a < 0 || b < 0 || a >= N || b >= N)
            return fail(CLOTH_EINVAL, "spring " + std::to_string(s) + " end out of range");
        if (a == b) return fail(CLOTH_EINVAL, "spring " + std::to_string(s) + " joins a node to itself");
        if (!(in.rest[s] > 0.0f) || !std::isfinite(in.rest[s]))
            return fail(CLOTH_EINVAL, "spring " + std::to_string(s) + " rest length must be > 0");
        if (!(in.k[s] >= 0.0f) || !std::isfinite(in.k[s]) || !(in.c[s] >= 0.0f) ||
            !std::isfinite(in.c[s]))
            return fail(CLOTH_EINVAL, "spring " + std::to_string(s) + " needs finite k, c >= 0");
    }
    if (in.n_verts < 0 || in.n_tris < 0) return fail(CLOTH_EINVAL, "negative surface size");
    if (in.n_tris > 0 && (!in.verts || !in.tris || in.n_verts <= 0))
        return fail(CLOTH_EINVAL, "verts and tris are required when n_tris > 0");
    for (long long i = 0; i < 3LL * in.n_verts; ++i)
        if (!std::isfinite(in.verts[i])) return fail(CLOTH_EINVAL, "non-finite surface vertex");
    for (int t = 0; t < in.n_tris; ++t) {
        int id[3];
        for (int q = 0; q < 3; ++q) {
            id[q] = in.tris[3 * t + q];
            if (id[q] < 0 || id[q] >= in.n_verts)
                return fail(CLOTH_EINVAL, "triangle " + std::to_string(t) + " vertex out of range");
        }
        const float* A = in.verts + 3 * id[0];
        const float* B = in.verts + 3 * id[1];
        const float* C = in.verts + 3 * id[2];
        const double e1[3] = {(double)B[0] - A[0], (double)B[1] - A[1], (double)B[2] - A[2]};
        const double e2[3] = {(double)C[0] - A[0], (double)C[1] - A[1], (double)C[2] - A[2]};
        const double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                             e1[0] * e2[1] - e1[1] * e2[0]};
        if (!(n[0] * n[0] + n[1] * n[1] + n[2] * n[2] > 0.0))
            return fail(CLOTH_EINVAL, "triangle " + std::to_string(t) + " has zero area");
    }
    return CLOTH_OK;
}

int validate_params(const cloth_params* p) {
    if (!p) return fail(CLOTH_EINVAL, "params are required");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(p->gravity[a])) return fail(CLOTH_EINVAL, "non-finite gravity");
    if (!(p->thickness >= 0.0f) || !std::isfinite(p->thickness))
        return fail(CLOTH_EINVAL, "thickness must be finite and >= 0");
    if (!(p->restitution >= 0.0f && p->restitution <= 1.0f))
        return fail(CLOTH_EINVAL, "restitution must be in [0, 1]");
    if (!std::isfinite(p->cell_size)) return fail(CLOTH_EINVAL, "non-finite cell_size");
    return CLOTH_OK;
}

// Stability bounds at the input configuration: w^2 and g are the largest Gershgorin row sums
// of M^-1 K and M^-1 C, with K and C assembled from 3x3 blocks k u u^T (c u u^T) per spring.
// Row (i, a) of K holds the diagonal block sum and one off-diagonal block per spring, so its
// absolute row sum is sum_s 2 k_s |u_a| (|u_x| + |u_y| + |u_z|).
void stability_bounds(const ClothHostInput& in, double* omega2, double* gamma) {
    const long long N = (long long)in.nx * in.ny;
    std::vector<double> rk(3 * N, 0.0), rc(3 * N, 0.0);
    for (int s = 0; s < in.n_springs; ++s) {
        const int a = in.ends[2 * s], b = in.ends[2 * s + 1];
        double d[3], l2 = 0.0;
        for (int q = 0; q < 3; ++q) {
            d[q] = (double)in.x0[3 * b + q] - in.x0[3 * a + q];
            l2 += d[q] * d[q];
        }
        const double l = std::sqrt(l2);
        double u[3] = {1.0, 0.0, 0.0};
        if (l > 0) {
            for (int q = 0; q < 3; ++q) u[q] = d[q] / l;
        }
        const double l1 = std::fabs(u[0]) + std::fabs(u[1]) + std::fabs(u[2]);
        for (int q = 0; q < 3; ++q) {
            const double vk = 2.0 * in.k[s] * std::fabs(u[q]) * l1;
            const double vc = 2.0 * in.c[s] * std::fabs(u[q]) * l1;
            rk[3 * a + q] += vk;
            rk[3 * b + q] += vk;
            rc[3 * a + q] += vc;
            rc[3 * b + q] += vc;
        }
    }
    double w2 = 0.0, g = 0.0;
    for (long long i = 0; i < N; ++i) {
        if (in.pinned && in.pinned[i]) continue;
        const double wi = 1.0 / (double)in.mass[i];
        for (int q = 0; q < 3; ++q) {
            w2 = std::max(w2, wi * rk[3 * i + q]);
            g = std::max(g, wi * rc[3 * i + q]);
        }
    }
    *omega2 = w2;
    *gamma = g;
}

bool unstable(double omega2, double gamma, double h) {
    return omega2 * h * h + 2.0 * gamma * h >= 4.0;
}

// Host-side cloth arrays in internal order.
int build_cloth_host(const ClothHostInput& in, ClothHost* out) {
    const int N = in.nx * in.ny;
    out->n = N;
    out->order = tile_order(in.nx, in.ny);
    out->slot.assign(N, 0);
    for (int p = 0; p < N; ++p) out->slot[out->order[p]] = p;
    out->ld = N;
    out->x.assign(3 * (size_t)N, 0.0f);
    out->v.assign(3 * (size_t)N, 0.0f);
    out->w.assign(N, 0.0f);
    for (int p = 0; p < N; ++p) {
        const int id = out->order[p];
        for (int q = 0; q < 3; ++q) {
            out->x[(size_t)q * N + p] = in.x0[3 * (size_t)id + q];
            out->v[(size_t)q * N + p] = in.v0 ? in.v0[3 * (size_t)id + q] : 0.0f;
        }
        const bool pin = in.pinned && in.pinned[id];
        out->w[p] = pin ? 0.0f : 1.0f / in.mass[id];
    }
    // incidences per internal node, sorted by (neighbour slot, spring id)
    std::vector<int> deg(N, 0);
    for (int s = 0; s < in.n_springs; ++s) {
        ++deg[out->slot[in.ends[2 * s]]];
        ++deg[out->slot[in.ends[2 * s + 1]]];
    }
    std::vector<int> start(N + 1, 0);
    for (int p = 0; p < N; ++p) start[p + 1] = start[p] + deg[p];
    std::vector<std::pair<long long, int>> inc(start[N]);  // (nbr slot << 32 | spring, code)
    std::vector<int> fill(N, 0);
    for (int s = 0; s < in.n_springs; ++s) {
        const int pa = out->slot[in.ends[2 * s]], pb = out->slot[in.ends[2 * s + 1]];
        inc[start[pa] + fill[pa]++] = {((long long)pb << 32) | (unsigned)s, s};
        inc[start[pb] + fill[pb]++] = {((long long)pa << 32) | (unsigned)s, ~s};
    }
    for (int p = 0; p < N; ++p) std::sort(inc.begin() + start[p], inc.begin() + start[p + 1]);
    const int n_slices = (N + 63) / 64;
    out->deg = deg;
    out->slice_ptr.assign(n_slices + 1, 0);
    for (int sl = 0; sl < n_slices; ++sl) {
        int mx = 0;
        for (int p = sl * 64; p < std::min(N, sl * 64 + 64); ++p) mx = std::max(mx, deg[p]);
        out->slice_ptr[sl + 1] = out->slice_ptr[sl] + mx * 64;
    }
    const size_t M = (size_t)out->slice_ptr[n_slices];
    out->nbr.assign(M, 0);
    out->ik.assign(M, 0.0f);
    out->ic.assign(M, 0.0f);
    out->il.assign(M, 1.0f);
    out->inc_spring.assign(M, 0);
    for (int p = 0; p < N; ++p) {
        const size_t base = (size_t)out->slice_ptr[p >> 6] + (p & 63);
        for (int r = 0; r < deg[p]; ++r) {
            const auto& e = inc[start[p] + r];
            const int s = e.second >= 0 ? e.second : ~e.second;
            const size_t q = base + (size_t)r * 64;
            out->nbr[q] = (int)(e.first >> 32);
            out->ik[q] = in.k[s];
            out->ic[q] = in.c[s];
            out->il[q] = in.rest[s];
            out->inc_spring[q] = e.second;
        }
        // padding slots point at the node itself with zero stiffness (never read)
        for (int r = deg[p]; r < (out->slice_ptr[(p >> 6) + 1] - out->slice_ptr[p >> 6]) / 64; ++r)
            out->nbr[base + (size_t)r * 64] = p;
    }
    return CLOTH_OK;
}

int upload_cloth(const ClothHost& h, DeviceArena& arena, hipStream_t stream, ClothDevice* d) {
    const int N = h.n;
    d->n = N;
    d->ld = h.ld;
    for (int b = 0; b < 2; ++b) {
        if (hipError_t e = arena.alloc(&d->x[b], 3 * (size_t)h.ld)) return hip_fail(e, "hipMalloc state");
        if (hipError_t e = arena.alloc(&d->v[b], 3 * (size_t)h.ld)) return hip_fail(e, "hipMalloc state");
    }
    const size_t M = h.nbr.size();
    hipError_t e;
    if ((e = arena.alloc(&d->w, (size_t)N)) || (e = arena.alloc(&d->deg, (size_t)N)) ||
        (e = arena.alloc(&d->slice_ptr, h.slice_ptr.size())) || (e = arena.alloc(&d->nbr, M)) ||
        (e = arena.alloc(&d->ik, M)) || (e = arena.alloc(&d->ic, M)) ||
        (e = arena.alloc(&d->il, M)) || (e = arena.alloc(&d->inc_spring, M)))
        return hip_fail(e, "hipMalloc cloth arrays");
    struct Cp {
        void* dst;
        const void* src;
        size_t bytes;
    } cps[] = {
        {d->x[0], h.x.data(), h.x.size() * 4},
        {d->v[0], h.v.data(), h.v.size() * 4},
        {d->w, h.w.data(), h.w.size() * 4},
        {d->deg, h.deg.data(), h.deg.size() * 4},
        {d->slice_ptr, h.slice_ptr.data(), h.slice_ptr.size() * 4},
        {d->nbr, h.nbr.data(), M * 4},
        {d->ik, h.ik.data(), M * 4},
        {d->ic, h.ic.data(), M * 4},
        {d->il, h.il.data(), M * 4},
        {d->inc_spring, h.inc_spring.data(), M * 4},
    };
    for (auto& c : cps)
        if (c.bytes)
            if ((e = hipMemcpyAsync(c.dst, c.src, c.bytes, hipMemcpyHostToDevice, stream)))
                return hip_fail(e, "upload cloth");
    d->cur = 0;
    return CLOTH_OK;
}

ClothView ClothDevice::view() const {
    ClothView v;
    v.n = n;
    v.ld = ld;
    v.w = w;
    v.deg = deg;
    v.slice_ptr = slice_ptr;
    v.nbr = nbr;
    v.ik = ik;
    v.ic = ic;
    v.il = il;
    v.inc_spring = inc_spring;
    return v;
}

// Uniform grid over the surface: origin fl32(min vertex) - thickness, cells of edge
// cell_size, dims ceil((max vertex + thickness - origin) / cell_size) per axis.
int build_surface(const ClothHostInput& in, const cloth_params& p, DeviceArena& arena,
                  hipStream_t stream, SurfaceDevice* sd) {
    sd->view = SurfaceView{};
    if (!(p.thickness > 0.0f) || in.n_tris == 0) return CLOTH_OK;
    const int T = in.n_tris, Vn = in.n_verts;
    double cell = p.cell_size;
    if (!(cell > 0.0)) {
        // 2 x mean length of the unique edges
        std::vector<std::pair<int, int>> edges;
        edges.reserve(3 * (size_t)T);
        for (int t = 0; t < T; ++t)
            for (int q = 0; q < 3; ++q) {
                int a = in.tris[3 * t + q], b = in.tris[3 * t + (q + 1) % 3];
                edges.emplace_back(std::min(a, b), std::max(a, b));
            }
        std::sort(edges.begin(), edges.end());
        edges.erase(std::unique(edges.begin(), edges.end()), edges.end());
        double sum = 0.0;
        for (auto& e : edges) {
            double l2 = 0.0;
            for (int q = 0; q < 3; ++q) {
                double dd = (double)in.verts[3 * e.second + q] - in.verts[3 * e.first + q];
                l2 += dd * dd;
            }
            sum += std::sqrt(l2);
        }
        cell = (double)(float)(2.0 * sum / (double)edges.size());
    }
    float vmin[3] = {INFINITY, INFINITY, INFINITY}, vmax[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = 0; i < Vn; ++i)
        for (int q = 0; q < 3; ++q) {
            vmin[q] = std::min(vmin[q], in.verts[3 * i + q]);
            vmax[q] = std::max(vmax[q], in.verts[3 * i + q]);
        }
    SurfaceView& sv = sd->view;
    long long cells = 1;
    for (int q = 0; q < 3; ++q) {
        sv.org[q] = vmin[q] - p.thickness;
        const double span = ((double)vmax[q] + p.thickness - (double)sv.org[q]) / cell;
        sv.dim[q] = (int)std::max(1.0, std::ceil(span));
        cells *= sv.dim[q];
        if (sv.dim[q] > (1 << 20)) return fail(CLOTH_ENOMEM, "grid too fine for the surface; raise cell_size");
    }
    if (cells > (1LL << 27)) return fail(CLOTH_ENOMEM, "grid too fine for the surface; raise cell_size");
    sv.inv_cell = (float)(1.0 / cell);
    sv.thickness = p.thickness;
    sv.thickness2 = p.thickness * p.thickness;
    sv.n_tris = T;
    sd->cell = cell;
    sd->n_cells = cells;

    hipError_t e;
    float* d_verts = nullptr;
    int* d_tris = nullptr;
    unsigned long long* d_total = nullptr;
    float4 *box_lo, *box_hi, *geo;
    if ((e = arena.alloc(&d_verts, 3 * (size_t)Vn)) || (e = arena.alloc(&d_tris, 3 * (size_t)T)) ||
        (e = arena.alloc(&d_total, 1)) || (e = arena.alloc(&box_lo, (size_t)T)) ||
        (e = arena.alloc(&box_hi, (size_t)T)) || (e = arena.alloc(&geo, 4 * (size_t)T)))
        return hip_fail(e, "hipMalloc surface");
    if ((e = hipMemcpyAsync(d_verts, in.verts, 12 * (size_t)Vn, hipMemcpyHostToDevice, stream)) ||
        (e = hipMemcpyAsync(d_tris, in.tris, 12 * (size_t)T, hipMemcpyHostToDevice, stream)) ||
        (e = hipMemsetAsync(d_total, 0, 8, stream)))
        return hip_fail(e, "upload surface");
    if ((e = launch_tri_prep(T, d_verts, d_tris, sv.thickness, sv.org, sv.inv_cell, sv.dim, box_lo,
                             box_hi, geo, d_total, stream)))
        return hip_fail(e, "triangle prep");
    unsigned long long total = 0;
    if ((e = hipMemcpyAsync(&total, d_total, 8, hipMemcpyDeviceToHost, stream)) ||
        (e = hipStreamSynchronize(stream)))
        return hip_fail(e, "read reference count");
    if (total > (1ULL << 30)) return fail(CLOTH_ENOMEM, "too many grid references; raise cell_size");
    uint32_t *counts, *cell_start, *refs, *tmp;
    const size_t C = (size_t)cells;
    if ((e = arena.alloc(&counts, C)) || (e = arena.alloc(&cell_start, C + 1)) ||
        (e = arena.alloc(&refs, (size_t)total)) || (e = arena.alloc(&tmp, scan_tmp_words(C))))
        return hip_fail(e, "hipMalloc grid");
    if ((e = hipMemsetAsync(counts, 0, 4 * C, stream)) ||
        (e = launch_grid_count(T, box_lo, box_hi, sv.org, sv.inv_cell, sv.dim, counts, stream)) ||
        (e = scan_exclusive_u32(counts, cell_start, C, tmp, stream)) ||
        (e = hipMemsetAsync(counts, 0, 4 * C, stream)) ||
        (e = launch_grid_fill(T, box_lo, box_hi, sv.org, sv.inv_cell, sv.dim, cell_start, counts,
                              refs, stream)) ||
        (e = launch_grid_sort((int)C, cell_start, refs, stream)) || (e = hipStreamSynchronize(stream)))
        return hip_fail(e, "grid build");
    arena.free_one(counts);
    arena.free_one(tmp);
    arena.free_one(d_verts);
    arena.free_one(d_tris);
    arena.free_one(d_total);
    sv.cell_start = cell_start;
    sv.refs = refs;
    sv.box_lo = box_lo;
    sv.box_hi = box_hi;
    sv.geo = geo;
    sd->n_refs = (long long)total;
    return CLOTH_OK;
}

}  // namespace cloth

// ------------------------------------------------------------------ the handle

struct cloth_sim {
    ClothHostInput shape;  // sizes only (pointers cleared after create)
    cloth_params p{};
    hipStream_t stream = nullptr;
    ClothHost host;
    ClothDevice dev;
    SurfaceDevice surf;
    DeviceArena arena;
    int* nan_flag = nullptr;
    double omega2 = 0.0, gamma = 0.0;
    int block = 256;
};

extern "C" {

int cloth_create(int nx, int ny, const float* x0, const float* v0, const float* mass,
                 const unsigned char* pinned, int n_springs, const int* ends, const float* rest,
                 const float* k, const float* c, int n_verts, const float* verts, int n_tris,
                 const int* tris, const cloth_params* p, void* hip_stream, cloth_sim** out) {
    if (!out) return fail(CLOTH_EINVAL, "out is NULL");
    *out = nullptr;
    ClothHostInput in{nx, ny, x0, v0, mass, pinned, n_springs, ends, rest, k, c, n_verts, verts,
                      n_tris, tris};
    int st;
    if ((st = validate_params(p)) || (st = validate_cloth(in))) return st;
    cloth_sim* s = new (std::nothrow) cloth_sim();
    if (!s) return fail(CLOTH_ENOMEM, "host allocation failed");
    s->p = *p;
    s->stream = (hipStream_t)hip_stream;
    try {
        st = build_cloth_host(in, &s->host);
        if (st == CLOTH_OK) stability_bounds(in, &s->omega2, &s->gamma);
    } catch (const std::bad_alloc&) {
        st = fail(CLOTH_ENOMEM, "host allocation failed");
    }
    if (st == CLOTH_OK) st = upload_cloth(s->host, s->arena, s->stream, &s->dev);
    if (st == CLOTH_OK) st = build_surface(in, s->p, s->arena, s->stream, &s->surf);
    if (st == CLOTH_OK) {
        hipError_t e;
        if ((e = s->arena.alloc(&s->nan_flag, 1)) ||
            (e = hipMemsetAsync(s->nan_flag, 0, 4, s->stream)) || (e = hipStreamSynchronize(s->stream)))
            st = hip_fail(e, "create");
    }
    if (st != CLOTH_OK) {
        (void)hipStreamSynchronize(s->stream);
        delete s;
        return st;
    }
    s->shape = in;
    s->shape.x0 = s->shape.v0 = s->shape.mass = s->shape.rest = s->shape.k = s->shape.c = nullptr;
    s->shape.verts = nullptr;
    s->shape.pinned = nullptr;
    s->shape.ends = s->shape.tris = nullptr;
    // host staging copies are no longer needed except the order maps
    s->host.release_arrays();
    *out = s;
    return CLOTH_OK;
}

int cloth_step(cloth_sim* s, float dt, int n_substeps, int n_steps) {
    if (!s) return fail(CLOTH_EINVAL, "NULL handle");
    if (!(dt > 0.0f) || !std::isfinite(dt)) return fail(CLOTH_EINVAL, "dt must be positive and finite");
    if (n_substeps < 1 || n_steps < 0) return fail(CLOTH_EINVAL, "n_substeps >= 1 and n_steps >= 0");
    const float h = dt / (float)n_substeps;
    if (!(s->p.flags & CLOTH_F_NO_STABILITY_CHECK) && unstable(s->omega2, s->gamma, h))
        return fail(CLOTH_EUNSTABLE, "substep h = " + std::to_string(h) +
                                         " s exceeds the explicit stability bound (omega^2 = " +
                                         std::to_string(s->omega2) + ", gamma = " +
                                         std::to_string(s->gamma) + "); use more substeps");
    StepParams sp;
    sp.h = h;
    for (int q = 0; q < 3; ++q) sp.g[q] = s->p.gravity[q];
    sp.restitution = s->p.restitution;
    sp.check_nan = (s->p.flags & CLOTH_F_CHECK_NAN) ? 1 : 0;
    sp.nan_flag = s->nan_flag;
    const ClothView cv = s->dev.view();
    const long long total = (long long)n_steps * n_substeps;
    for (long long it = 0; it < total; ++it) {
        const int src = s->dev.cur, dst = src ^ 1;
        hipError_t e = launch_substep(cv, s->surf.view, sp, s->dev.x[src], s->dev.v[src],
                                      s->dev.x[dst], s->dev.v[dst], s->block, s->stream);
        if (e != hipSuccess) return hip_fail(e, "substep launch");
        s->dev.cur = dst;
    }
    return CLOTH_OK;
}

int cloth_read_state(const cloth_sim* s, float* x_out, float* v_out) {
    if (!s || !x_out) return fail(CLOTH_EINVAL, "NULL argument");
    const int N = s->dev.n, ld = s->dev.ld;
    std::vector<float> xs(3 * (size_t)ld), vs(v_out ? 3 * (size_t)ld : 0);
    int flag = 0;
    hipError_t e;
    if ((e = hipMemcpyAsync(xs.data(), s->dev.x[s->dev.cur], 12 * (size_t)ld, hipMemcpyDeviceToHost,
                            s->stream)))
        return hip_fail(e, "read state");
    if (v_out && (e = hipMemcpyAsync(vs.data(), s->dev.v[s->dev.cur], 12 * (size_t)ld,
                                     hipMemcpyDeviceToHost, s->stream)))
        return hip_fail(e, "read state");
    if ((e = hipMemcpyAsync(&flag, s->nan_flag, 4, hipMemcpyDeviceToHost, s->stream)) ||
        (e = hipStreamSynchronize(s->stream)))
        return hip_fail(e, "read state");
    for (int p = 0; p < N; ++p) {
        const int id = s->host.order[p];
        for (int q = 0; q < 3; ++q) {
            x_out[3 * (size_t)id + q] = xs[(size_t)q * ld + p];
            if (v_out) v_out[3 * (size_t)id + q] = vs[(size_t)q * ld + p];
        }
    }
    if ((s->p.flags & CLOTH_F_CHECK_NAN) && flag)
        return fail(CLOTH_ENAN, "a non-finite value appeared in the state");
    return CLOTH_OK;
}

int cloth_write_state(cloth_sim* s, const float* x, const float* v) {
    if (!s || !x) return fail(CLOTH_EINVAL, "NULL argument");
    const int N = s->dev.n, ld = s->dev.ld;
    std::vector<float> xs(3 * (size_t)ld, 0.0f), vs(3 * (size_t)ld, 0.0f);
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
    out[0] = s->dev.n;
    out[1] = s->shape.n_springs;
    out[2] = s->surf.view.n_tris;
    out[3] = s->surf.n_cells;
    out[4] = s->surf.n_refs;
    for (int q = 0; q < 3; ++q) out[5 + q] = s->surf.view.n_tris ? s->surf.view.dim[q] : 0;
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
    if (s->surf.view.n_tris == 0) return fail(CLOTH_EINVAL, "collision is disabled for this handle");
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
    if ((e = hipMemcpyAsync(d_p, soa.data(), 12 * n, hipMemcpyHostToDevice, s->stream)) ||
        (e = launch_candidates_count(n_points, n_points, d_p, s->surf.view, d_cnt, s->stream)) ||
        (e = scan_exclusive_u32(d_cnt, d_off, n, d_scan, s->stream)) ||
        (e = hipMemcpyAsync(&total, d_off + n, 4, hipMemcpyDeviceToHost, s->stream)) ||
        (e = hipStreamSynchronize(s->stream)))
        return hip_fail(e, "candidate count");
    *n_out = total;
    if (total == 0 || cap == 0) return CLOTH_OK;
    int* d_pairs;
    if ((e = tmp.alloc(&d_pairs, 2 * (size_t)total))) return hip_fail(e, "hipMalloc pairs");
    const size_t ncopy = (size_t)std::min<long long>(cap, total);
    if ((e = launch_candidates_write(n_points, n_points, d_p, s->surf.view, d_off, d_pairs, s->stream)) ||
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

}  // extern "C"
