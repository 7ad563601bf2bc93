// Host-side building blocks of a simulation handle: error plumbing, input validation, the
// internal node order, the sliced CSR incidence build, the stability bound and the surface
// grid build.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/cloth.h"
#include "cloth_internal.h"
#include "host_common.h"

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

// Scratch words of scan_exclusive_u32 over n entries: the tile totals and their offsets at
// every level of the recursion.
size_t scan_tmp_words(size_t n) {
    const size_t m = n + 1;
    const size_t nb = (m + kScanTile - 1) / kScanTile;
    if (nb <= 1) return 1;
    return nb + (nb + 1) + scan_tmp_words(nb);
}

// LDS of one tile workgroup: two copies (ping-pong) of the region's x and v, 12 floats per
// node, plus the hit lists of its wavefronts.
size_t tile_lds_bytes(int rmax, int block, int hit_slots) {
    return (size_t)12 * sizeof(float) * (size_t)rmax + (size_t)(block / 64) * wave_query_lds(hit_slots);
}

void DeviceArena::free_one(void* p) {
    if (!p) return;
    auto it = std::find(ptrs.begin(), ptrs.end(), p);
    if (it != ptrs.end()) {
        (void)hipFree(p);
        ptrs.erase(it);
    }
}

// Internal node order: the nx-by-ny grid is cut into 8x8 tiles (narrower in the last tile
// column, shorter in the last tile row), the tiles are taken row by row, and nodes are
// row-major within a tile.  A wavefront of 64 consecutive slots is then one 8x8 patch, and
// the slot of node (row, column) is plain arithmetic on the grid shape (see k_grid).
std::vector<std::pair<int, int>> tile_list(int nx, int ny) {
    const int T = 8;
    const int tx = (nx + T - 1) / T, ty = (ny + T - 1) / T;
    std::vector<std::pair<int, int>> out;
    out.reserve((size_t)tx * ty);
    for (int j = 0; j < ty; ++j)
        for (int i = 0; i < tx; ++i) out.emplace_back(i, j);
    return out;
}

std::vector<int> tile_order(int nx, int ny) {
    const int T = 8;
    std::vector<int> order;
    order.reserve((size_t)nx * ny);
    for (const auto& [ti, tj] : tile_list(nx, ny))
        for (int i = tj * T; i < std::min(ny, tj * T + T); ++i)
            for (int j = ti * T; j < std::min(nx, ti * T + T); ++j) order.push_back(i * nx + j);
    return order;
}

// Grid stencil of a handle whose cloths are all grids (sides below 2^15) with springs only
// between nodes at the twelve offsets (row, column) of the stencil, one spring per node and
// offset at most.  code[d * ld + p]: the spring from slot p to its neighbour in direction d,
// or -1.  tiles: per 8x8 tile of the handle, in slot order, its cloth as (first slot,
// nx | ny << 16, first tile of the cloth, cloth index).
bool build_stencil(const std::vector<StencilCloth>& cloths, const std::vector<int>& ends,
                   const std::vector<int>& slot, int ld, std::vector<int>* code,
                   std::vector<int4>* tiles) {
    static const int dr[kStencilDirs] = {-2, -1, -1, -1, 0, 0, 0, 0, 1, 1, 1, 2};
    static const int dc[kStencilDirs] = {0, -1, 0, 1, -2, -1, 1, 2, -1, 0, 1, 0};
    int dir_of[5][5];
    for (auto& row : dir_of)
        for (int& v : row) v = -1;
    for (int d = 0; d < kStencilDirs; ++d) dir_of[dr[d] + 2][dc[d] + 2] = d;
    code->assign((size_t)kStencilDirs * ld, -1);
    tiles->clear();
    for (size_t g = 0; g < cloths.size(); ++g) {
        const StencilCloth& c = cloths[g];
        if (c.nx >= (1 << 15) || c.ny >= (1 << 15)) return false;
        for (int s = c.spring_off; s < c.spring_off + c.n_springs; ++s) {
            const int a = ends[2 * (size_t)s] - c.node_off, b = ends[2 * (size_t)s + 1] - c.node_off;
            const int rr = b / c.nx - a / c.nx, cc = b % c.nx - a % c.nx;
            if (rr < -2 || rr > 2 || cc < -2 || cc > 2) return false;
            const int da = dir_of[rr + 2][cc + 2], db = dir_of[2 - rr][2 - cc];
            if (da < 0) return false;
            int& ca = (*code)[(size_t)da * ld + slot[c.node_off + a]];
            int& cb = (*code)[(size_t)db * ld + slot[c.node_off + b]];
            if (ca >= 0 || cb >= 0) return false;  // a second spring at the same offset
            ca = s;
            cb = s;
        }
        // the stencil kernel computes slots from the grid shape: they must be these
        for (int gr = 0; gr < c.ny; ++gr)
            for (int gc = 0; gc < c.nx; ++gc) {
                const int tr = gr >> 3, tc = gc >> 3;
                const int h = std::min(8, c.ny - 8 * tr), w = std::min(8, c.nx - 8 * tc);
                const int want = c.slot_off + 8 * c.nx * tr + 8 * h * tc + (gr & 7) * w + (gc & 7);
                if (slot[c.node_off + gr * c.nx + gc] != want) return false;
            }
        const int first = (int)tiles->size();
        const size_t n_t = tile_list(c.nx, c.ny).size();
        for (size_t q = 0; q < n_t; ++q)
            tiles->push_back(make_int4(c.slot_off, c.nx | (c.ny << 16), first, (int)g));
    }
    return true;
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
    if (p->flags & ~(CLOTH_F_CHECK_NAN | CLOTH_F_NO_STABILITY_CHECK | CLOTH_F_NARROW_MT))
        return fail(CLOTH_EINVAL, "unknown flag");
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
int build_cloth_host(const ClothHostInput& in, ClothHost* out, const std::vector<int>* order,
                     const std::vector<int>* segs) {
    const int N = in.nx * in.ny;
    out->n = N;
    out->order = order ? *order : tile_order(in.nx, in.ny);
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
    // incidences per internal node, sorted by (neighbour node id, spring id): on a grid cloth
    // that is the order of the offsets (row, column) of the neighbours, the same for every
    // node, so the stencil kernel sums in this order too
    std::vector<int> deg(N, 0);
    for (int s = 0; s < in.n_springs; ++s) {
        ++deg[out->slot[in.ends[2 * s]]];
        ++deg[out->slot[in.ends[2 * s + 1]]];
    }
    std::vector<int> start(N + 1, 0);
    for (int p = 0; p < N; ++p) start[p + 1] = start[p] + deg[p];
    struct Inc {
        long long key;  // neighbour id << 32 | spring
        int nbr;        // neighbour slot
        int code;       // spring, ~spring at its second end
        bool operator<(const Inc& o) const { return key < o.key; }
    };
    std::vector<Inc> inc(start[N]);
    std::vector<int> fill(N, 0);
    for (int s = 0; s < in.n_springs; ++s) {
        const int ia = in.ends[2 * s], ib = in.ends[2 * s + 1];
        const int pa = out->slot[ia], pb = out->slot[ib];
        inc[start[pa] + fill[pa]++] = {((long long)ib << 32) | (unsigned)s, pb, s};
        inc[start[pb] + fill[pb]++] = {((long long)ia << 32) | (unsigned)s, pa, ~s};
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
    out->inc_spring.assign(M, 0);
    for (int p = 0; p < N; ++p) {
        const size_t base = (size_t)out->slice_ptr[p >> 6] + (p & 63);
        for (int r = 0; r < deg[p]; ++r) {
            const auto& e = inc[start[p] + r];
            const size_t q = base + (size_t)r * 64;
            out->nbr[q] = e.nbr;
            out->inc_spring[q] = e.code;
        }
        // padding slots point at the node itself and at spring 0 (never read)
        for (int r = deg[p]; r < (out->slice_ptr[(p >> 6) + 1] - out->slice_ptr[p >> 6]) / 64; ++r)
            out->nbr[base + (size_t)r * 64] = p;
    }
    param_table(in.k, in.c, in.rest, in.n_springs, segs, &out->ptab, &out->spring_entry,
                &out->tab_span);
    return CLOTH_OK;
}

void param_table(const float* k, const float* c, const float* rest, int S,
                 const std::vector<int>* segs, std::vector<float4>* tab,
                 std::vector<int>* entry, int* span) {
    struct Key {
        uint32_t a, b, c;
        bool operator==(const Key& o) const { return a == o.a && b == o.b && c == o.c; }
    };
    struct Hash {
        size_t operator()(const Key& x) const {
            uint64_t h = x.a * 0x9e3779b97f4a7c15ULL;
            h ^= (h >> 29) + x.b * 0xbf58476d1ce4e5b9ULL;
            h ^= (h >> 31) + x.c * 0x94d049bb133111ebULL;
            return (size_t)(h ^ (h >> 32));
        }
    };
    std::unordered_map<Key, int, Hash> index;
    tab->clear();
    entry->assign((size_t)S, 0);
    *span = 0;
    size_t seg = 1, first = 0;  // the current segment ends before (*segs)[seg]
    for (int s = 0; s < S; ++s) {
        if (segs && seg < segs->size() && s >= (*segs)[seg]) {
            while (seg < segs->size() && s >= (*segs)[seg]) ++seg;
            *span = std::max(*span, (int)(tab->size() - first));
            first = tab->size();
            index.clear();
        }
        Key key;
        std::memcpy(&key.a, k + s, 4);
        std::memcpy(&key.b, c + s, 4);
        std::memcpy(&key.c, rest + s, 4);
        auto it = index.find(key);
        if (it == index.end()) {
            it = index.emplace(key, (int)tab->size()).first;
            tab->push_back(make_float4(k[s], c[s], rest[s], 0.0f));
        }
        (*entry)[s] = it->second;
    }
    *span = std::max(*span, (int)(tab->size() - first));
}

std::vector<int> segment_bases(const std::vector<int>& segs, const std::vector<int>& entry) {
    std::vector<int> b;
    for (size_t g = 0; g + 1 < segs.size(); ++g)
        b.push_back(segs[g] < segs[g + 1] ? entry[(size_t)segs[g]] : 0);
    return b;
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
    const size_t S = h.spring_entry.size();
    d->n_springs = (int)S;
    hipError_t e;
    // the table has room for one entry per spring, so a parameter update never moves it
    // (captured graphs keep its address)
    if ((e = arena.alloc(&d->w, (size_t)N)) || (e = arena.alloc(&d->deg, (size_t)N)) ||
        (e = arena.alloc(&d->slice_ptr, h.slice_ptr.size())) || (e = arena.alloc(&d->inc2, M)) ||
        (e = arena.alloc(&d->inc_spring, M)) || (e = arena.alloc(&d->ptab, std::max<size_t>(S, 1))) ||
        (e = arena.alloc(&d->spring_entry, std::max<size_t>(S, 1))) ||
        (e = arena.alloc(&d->n_tab, 1)))
        return hip_fail(e, "hipMalloc cloth arrays");
    std::vector<uint2> inc2(M);
    const int n_tab = h.tab_span;
    StreamFence fence{stream};
    for (size_t q = 0; q < M; ++q) {
        const int code = h.inc_spring[q];
        const int s = code >= 0 ? code : ~code;
        inc2[q] = make_uint2((uint32_t)h.nbr[q], S ? (uint32_t)h.spring_entry[s] : 0u);
    }
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
        {d->inc2, inc2.data(), M * sizeof(uint2)},
        {d->inc_spring, h.inc_spring.data(), M * 4},
        {d->ptab, h.ptab.data(), h.ptab.size() * sizeof(float4)},
        {d->spring_entry, h.spring_entry.data(), S * 4},
        {d->n_tab, &n_tab, sizeof(int)},
    };
    for (auto& c : cps)
        if (c.bytes)
            if ((e = hipMemcpyAsync(c.dst, c.src, c.bytes, hipMemcpyHostToDevice, stream)))
                return hip_fail(e, "upload cloth");
    // the packed records live on this stack frame: finish the copies before returning (the
    // fence covers the error returns)
    if ((e = hipStreamSynchronize(stream))) return hip_fail(e, "upload cloth");
    d->cur = 0;
    return CLOTH_OK;
}

GridView ClothDevice::grid_view() const {
    GridView g;
    g.n_tiles = n_tiles;
    g.one = one_cloth;
    g.tiles = tiles;
    g.idx = sten_idx;
    g.idx8 = sten_idx8;
    g.n_tab = this->n_tab;
    g.tab_cap = std::max(n_springs, 1);
    g.tab_base = tab_base;
    return g;
}

ClothView ClothDevice::view() const {
    ClothView v;
    v.n = n;
    v.ld = ld;
    v.w = w;
    v.deg = deg;
    v.slice_ptr = slice_ptr;
    v.inc2 = inc2;
    v.ptab = ptab;
    v.inc_spring = inc_spring;
    return v;
}

int upload_param_table(const std::vector<float4>& tab, const std::vector<int>& entry, int span,
                       const std::vector<int>& bases, ClothDevice* d, size_t n_inc,
                       uint2* plan_rec, const int* plan_sid, size_t n_plan, hipStream_t stream) {
    if (entry.size() != (size_t)d->n_springs || tab.size() > std::max<size_t>(entry.size(), 1))
        return fail(CLOTH_EINVAL, "parameter table does not match the springs");
    StreamFence fence{stream};
    hipError_t e;
    if ((tab.size() &&
         (e = hipMemcpyAsync(d->ptab, tab.data(), tab.size() * sizeof(float4),
                             hipMemcpyHostToDevice, stream))) ||
        (entry.size() && (e = hipMemcpyAsync(d->spring_entry, entry.data(), entry.size() * 4,
                                             hipMemcpyHostToDevice, stream))))
        return hip_fail(e, "upload parameter table");
    if (d->tab_base && bases.size() &&
        (e = hipMemcpyAsync(d->tab_base, bases.data(), bases.size() * 4, hipMemcpyHostToDevice,
                            stream)))
        return hip_fail(e, "upload parameter table");
    if (entry.size()) {
        if ((e = launch_set_entries(n_inc, d->inc_spring, 1, d->spring_entry, d->inc2, stream)))
            return hip_fail(e, "re-point incidence records");
        if (plan_rec && n_plan &&
            (e = launch_set_entries(n_plan, plan_sid, 0, d->spring_entry, plan_rec, stream)))
            return hip_fail(e, "re-point tile records");
        if (d->sten_code &&
            (e = launch_set_stencil_entries(d->ld, d->sten_code, d->spring_entry, d->slot_cloth,
                                            d->tab_base, d->sten_idx, d->sten_idx8, stream)))
            return hip_fail(e, "re-point stencil entries");
    }
    const int n_tab = span;
    if ((e = hipMemcpyAsync(d->n_tab, &n_tab, sizeof(int), hipMemcpyHostToDevice, stream)))
        return hip_fail(e, "upload parameter table");
    // the host vectors are the copies' sources: finish before returning
    if ((e = hipStreamSynchronize(stream))) return hip_fail(e, "upload parameter table");
    return CLOTH_OK;
}

constexpr size_t kRefPad = kRefRound;

// Uniform grid over the surface: origin fl32(min vertex) - thickness, cells of edge
// cell_size, dims floor((fl32(max vertex + thickness) - origin) / cell_size) + 1 per axis.
// The cell size is fixed when the surface is first built; origin, dims and every derived
// array are recomputed by each rebuild.
int build_surface(const ClothHostInput& in, const cloth_params& p, DeviceArena& arena,
                  hipStream_t stream, SurfaceDevice* sd) {
    sd->view = SurfaceView{};
    if (!(p.thickness > 0.0f) || in.n_tris == 0) return CLOTH_OK;
    const int T = in.n_tris, Vn = in.n_verts;
    StreamFence fence{stream};  // in.tris and in.verts are the caller's: copies finish here
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
    SurfaceView& sv = sd->view;
    sv.inv_cell = (float)(1.0 / cell);
    sv.thickness = p.thickness;
    sv.thickness2 = p.thickness * p.thickness;
    sv.n_tris = T;
    sd->cell = cell;
    sd->n_verts = Vn;
    hipError_t e;
    if ((e = arena.alloc(&sd->verts, 3 * (size_t)Vn)) || (e = arena.alloc(&sd->tris, 3 * (size_t)T)) ||
        (e = arena.alloc(&sd->total, 1)) || (e = arena.alloc(&sd->box_lo, (size_t)T)) ||
        (e = arena.alloc(&sd->box_hi, (size_t)T)) || (e = arena.alloc(&sd->geo, 3 * (size_t)T)) ||
        (e = arena.alloc(&sd->tri_v, 3 * (size_t)T)))
        return hip_fail(e, "hipMalloc surface");
    if ((e = hipMemcpyAsync(sd->tris, in.tris, 12 * (size_t)T, hipMemcpyHostToDevice, stream)))
        return hip_fail(e, "upload surface");
    return rebuild_surface(sd, in.verts, arena, stream);
}

int rebuild_surface(SurfaceDevice* sd, const float* verts, DeviceArena& arena,
                    hipStream_t stream) {
    SurfaceView& sv = sd->view;
    const int T = sv.n_tris, Vn = sd->n_verts;
    // verts is the caller's and `total` below lives here: the copies finish before any return
    unsigned long long total = 0;
    StreamFence fence{stream};
    float vmin[3] = {INFINITY, INFINITY, INFINITY}, vmax[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = 0; i < Vn; ++i)
        for (int q = 0; q < 3; ++q) {
            const float c = verts[3 * i + q];
            if (!std::isfinite(c)) return fail(CLOTH_EINVAL, "non-finite surface vertex");
            vmin[q] = std::min(vmin[q], c);
            vmax[q] = std::max(vmax[q], c);
        }
    float org[3];
    int dim[3];
    long long cells = 1;
    for (int q = 0; q < 3; ++q) {
        // origin at or below every inflated low corner; dims so the largest inflated high
        // corner maps to dim - 1 with the kernels' own FP32 formula floor((p - org) * inv)
        org[q] = vmin[q] - sv.thickness;
        const float hmax = vmax[q] + sv.thickness;
        volatile float diff = hmax - org[q];
        volatile float scaled = diff * sv.inv_cell;
        const double top = std::floor((double)scaled);
        if (!(top < (double)(1 << 20))) return fail(CLOTH_ENOMEM, "grid too fine for the surface; raise cell_size");
        dim[q] = (int)top + 1;
        cells *= dim[q];
    }
    if (cells > (1LL << 27)) return fail(CLOTH_ENOMEM, "grid too fine for the surface; raise cell_size");
    const size_t C = (size_t)cells;
    hipError_t e;
    sd->dirty = true;
    // every buffer is reused while it is large enough, so a moving surface reallocates only
    // when its grid or reference count grows
    if (C > sd->cap_cells) {
        if ((e = hipStreamSynchronize(stream))) return hip_fail(e, "grid resize");
        arena.free_one(sd->counts);
        arena.free_one(sd->cell_start);
        arena.free_one(sd->tmp);
        sd->counts = sd->cell_start = sd->tmp = nullptr;
        sd->cap_cells = 0;
        const size_t cap = C + C / 4;
        if ((e = arena.alloc(&sd->counts, cap)) || (e = arena.alloc(&sd->cell_start, cap + 1)) ||
            (e = arena.alloc(&sd->tmp, scan_tmp_words(cap))))
            return hip_fail(e, "hipMalloc grid");
        sd->cap_cells = cap;
    }
    for (int q = 0; q < 3; ++q) {
        sv.org[q] = org[q];
        sv.dim[q] = dim[q];
    }
    sd->n_cells = cells;
    if ((e = hipMemcpyAsync(sd->verts, verts, 12 * (size_t)Vn, hipMemcpyHostToDevice, stream)) ||
        (e = hipMemsetAsync(sd->total, 0, 8, stream)))
        return hip_fail(e, "upload surface");
    if ((e = launch_tri_prep(T, sd->verts, sd->tris, sv.thickness, sv.org, sv.inv_cell, sv.dim,
                             sd->box_lo, sd->box_hi, sd->geo, sd->tri_v, sd->total, stream)))
        return hip_fail(e, "triangle prep");
    if ((e = hipMemcpyAsync(&total, sd->total, 8, hipMemcpyDeviceToHost, stream)) ||
        (e = hipStreamSynchronize(stream)))
        return hip_fail(e, "read reference count");
    if (total > (1ULL << 30)) return fail(CLOTH_ENOMEM, "too many grid references; raise cell_size");
    if ((size_t)total + kRefPad > sd->cap_refs) {
        arena.free_one(sd->refs);
        arena.free_one(sd->ref_lo);
        arena.free_one(sd->ref_hi);
        arena.free_one(sd->ref_q);
        sd->refs = nullptr;
        sd->ref_lo = sd->ref_hi = nullptr;
        sd->ref_q = nullptr;
        sd->cap_refs = 0;
        const size_t cap = (size_t)total + (size_t)total / 4 + kRefPad;
        if ((e = arena.alloc(&sd->refs, cap)) || (e = arena.alloc(&sd->ref_lo, cap)) ||
            (e = arena.alloc(&sd->ref_hi, cap)) || (e = arena.alloc(&sd->ref_q, cap)))
            return hip_fail(e, "hipMalloc grid");
        sd->cap_refs = cap;
        // kRefPad entries after the last reference let the query loops load a round of
        // references without a bounds test (the loaded values past a cell's end are never
        // used, but a reference's triangle id may be followed): zeroed once here, every entry
        // past a later build's last reference holds zero or an earlier build's reference, so
        // always a valid triangle id
        if ((e = hipMemsetAsync(sd->refs, 0, 4 * cap, stream)) ||
            (e = hipMemsetAsync(sd->ref_lo, 0, sizeof(float4) * cap, stream)) ||
            (e = hipMemsetAsync(sd->ref_hi, 0, sizeof(float4) * cap, stream)) ||
            (e = hipMemsetAsync(sd->ref_q, 0, sizeof(uint4) * cap, stream)))
            return hip_fail(e, "grid build");
    }
    if ((e = hipMemsetAsync(sd->counts, 0, 4 * C, stream)) ||
        (e = launch_grid_count(T, sd->box_lo, sd->box_hi, sv.org, sv.inv_cell, sv.dim, sd->counts,
                               stream)) ||
        (e = scan_exclusive_u32(sd->counts, sd->cell_start, C, sd->tmp, stream)) ||
        (e = hipMemsetAsync(sd->counts, 0, 4 * C, stream)) ||
        (e = launch_grid_fill(T, sd->box_lo, sd->box_hi, sv.org, sv.inv_cell, sv.dim,
                              sd->cell_start, sd->counts, sd->refs, stream)) ||
        (e = launch_grid_finish((int)C, sv.org, sv.inv_cell, sv.dim, sd->cell_start, sd->refs,
                                sd->box_lo, sd->box_hi, sd->ref_lo, sd->ref_hi, sd->ref_q,
                                stream)))
        return hip_fail(e, "grid build");
    sv.cell_start = sd->cell_start;
    sv.refs = sd->refs;
    sv.ref_lo = sd->ref_lo;
    sv.ref_hi = sd->ref_hi;
    sv.ref_q = sd->ref_q;
    sv.box_lo = sd->box_lo;
    sv.box_hi = sd->box_hi;
    sv.geo = sd->geo;
    sv.tri_v = sd->tri_v;
    sd->n_refs = (long long)total;
    sd->dirty = false;
    return CLOTH_OK;
}

}  // namespace cloth
