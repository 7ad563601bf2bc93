// Triangle-triangle narrow phase (the extended Moller-Trumbore process of Sec. 3) as an
// alternative to the point-triangle proximity test.  A substep is two launches: the
// collision-free prediction of every node (forces and integration, into a scratch state),
// then four lanes per node (each scanning a quarter of the node's query cells) that find the
// node's contact set from the predictions of its cloth neighbours, and the response.
// Surface triangle t is a contact of node i when
//   (A) a cloth edge at i crosses t (oriented from the lower node id),
//   (B) an edge of t (oriented from the lower vertex id) crosses a cloth triangle at i, or
//   (C) i's path from its start position to its prediction crosses t.
// The cloth mesh is the grid's quads split along their (r, c)-(r+1, c+1) diagonals.
// Each segment test is preceded by exact-in-principle rejections (the segment's ends strictly
// on one side of the triangle's plane, or boxes that do not meet), which differ from the
// full test only at decision boundaries.  A crossing lies in the triangle, so the boxes
// tested are the triangle's own (the grid's boxes, grown by the thickness for the proximity
// query, shrunk back to the triangle plus a margin of a thousandth of the thickness, at
// least 1 um, far above the rounding of either box).  Candidates come from the grid cells
// covering the box of i's path, edges and triangles; a
// triangle listed in several of those cells is tested only in the first of them (the cell
// whose coordinates are the maxima of its own and the query's low cells), so each
// candidate is tested once, in a fixed order.  The response is the averaged push of Alg. 2:
// x = x* + mean_t (th - (x* - A_t).n_t) n_t, v = -restitution v*.
#include "cloth_device.h"
#include "cloth_internal.h"

namespace cloth {

namespace {

constexpr float kMtEps = 1e-7f;
constexpr float kMtBoxMargin = 1e-3f;  // of the thickness (see above)

__device__ __forceinline__ float3 f3(const float4& a) { return make_float3(a.x, a.y, a.z); }
__device__ __forceinline__ float3 sub3(float3 a, float3 b) {
    return make_float3(a.x - b.x, a.y - b.y, a.z - b.z);
}
__device__ __forceinline__ float dot3(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ float3 cross3(float3 a, float3 b) {
    return make_float3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

// Does segment S -> E cross triangle (V0, V1, V2)?  The six steps of the extended
// Moller-Trumbore process: direction r = d / |d|, h = r x e2, a = e1 . h (parallel when
// |a| < eps), u = (s . h) / a in [0, 1], v = (r . q) / a >= 0 with u + v <= 1, and the
// crossing distance t = (e2 . q) / a strictly inside (eps, |d|).  Kept out of line: it is
// called from 25 places per candidate.
__device__ __noinline__ bool mt_cross(float3 S, float3 E, float3 V0, float3 V1, float3 V2) {
    const float3 d = sub3(E, S);
    const float len2 = dot3(d, d);
    if (!(len2 > 0.0f)) return false;
    const float len = sqrtf(len2);
    const float3 r = make_float3(d.x / len, d.y / len, d.z / len);
    const float3 e1 = sub3(V1, V0), e2 = sub3(V2, V0);
    const float3 h = cross3(r, e2);
    const float a = dot3(e1, h);
    if (fabsf(a) < kMtEps) return false;
    const float f = 1.0f / a;
    const float3 s = sub3(S, V0);
    const float u = f * dot3(s, h);
    if (u < 0.0f || u > 1.0f) return false;
    const float3 q = cross3(s, e1);
    const float v = f * dot3(r, q);
    if (v < 0.0f || u + v > 1.0f) return false;
    const float t = f * dot3(e2, q);
    return kMtEps < t && t < len;
}

// False only when a and b are both strictly positive or both strictly negative.
__device__ __forceinline__ bool straddles(float a, float b) {
    return !((a > 0.0f && b > 0.0f) || (a < 0.0f && b < 0.0f));
}

__device__ __forceinline__ bool seg_meets_box(float3 a, float3 b, const float4& lo, const float4& hi) {
    return fmaxf(a.x, b.x) >= lo.x && fminf(a.x, b.x) <= hi.x && fmaxf(a.y, b.y) >= lo.y &&
           fminf(a.y, b.y) <= hi.y && fmaxf(a.z, b.z) >= lo.z && fminf(a.z, b.z) <= hi.z;
}

__device__ __forceinline__ bool tri_meets_box(float3 a, float3 b, float3 c, const float4& lo,
                                              const float4& hi) {
    return fmaxf(fmaxf(a.x, b.x), c.x) >= lo.x && fminf(fminf(a.x, b.x), c.x) <= hi.x &&
           fmaxf(fmaxf(a.y, b.y), c.y) >= lo.y && fminf(fminf(a.y, b.y), c.y) <= hi.y &&
           fmaxf(fmaxf(a.z, b.z), c.z) >= lo.z && fminf(fminf(a.z, b.z), c.z) <= hi.z;
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Candidates a lane lists in LDS before their triangles are loaded and tested, and
// reference boxes tested per round of loads.
constexpr int kMtSlots = 24;
constexpr int kMtRefRound = 8;
constexpr int kMtLanes = 4;  // lanes per node of the stepping kernel

// LANES lanes per node, in LANES consecutive wavefronts of a 256-thread workgroup: lane j
// takes the cells of the node's query box whose ordinal is j modulo LANES, and lanes 1 ..
// LANES - 1 add their contact sums to lane 0's through LDS, in that order (the debug form
// keeps one lane per node, so each node's ids are written by one thread in test order).
template <int LANES>
constexpr int mt_nodes_per_block() { return 256 / LANES; }

template <bool DEBUG, int LANES>
__global__ void __launch_bounds__(256)
    k_mt_collide(const ClothView cv, const StepParams sp, const int* __restrict__ order,
                 const int* __restrict__ slot, const int* __restrict__ node_group,
                 const int4* __restrict__ groups, const SurfaceView* __restrict__ svs,
                 const float* __restrict__ xs, const float* __restrict__ P, float* __restrict__ xd,
                 float* __restrict__ vd, int* __restrict__ counts, int* __restrict__ ids, int cap) {
    static_assert(LANES == 1 || LANES == 2 || LANES == 4, "1, 2 or 4 lanes per node");
    static_assert(!(DEBUG && LANES > 1), "the debug form runs one lane per node");
    constexpr bool SPLIT = LANES > 1;
    constexpr int kNodes = mt_nodes_per_block<LANES>();
    __shared__ uint32_t lists[4 * 64 * kMtSlots];   // each lane's list: every 64th word
    __shared__ float4 part[SPLIT ? LANES - 1 : 1][SPLIT ? kNodes : 1];  // lanes 1..: sums, counts
    uint32_t* list = lists + (threadIdx.x >> 6) * 64 * kMtSlots + (threadIdx.x & 63);
    const int lane = threadIdx.x & 63;
    const int share = SPLIT ? (threadIdx.x >> 6) % LANES : 0;  // this lane's share of the cells
    const int pair = SPLIT ? (threadIdx.x >> 6) / LANES * 64 + lane : 0;  // the node in part
    const int p = SPLIT ? blockIdx.x * kNodes + pair : blockIdx.x * blockDim.x + threadIdx.x;
    if (!SPLIT && p >= cv.n) return;
    const bool node = p < cv.n;  // (with SPLIT every thread reaches the barrier below)
    const int ld = cv.ld;
    const int pn = node ? p : 0;
    const float* Pv = P + 3 * (size_t)ld;
    float3 xp = make_float3(P[pn], P[ld + pn], P[2 * ld + pn]);
    float3 vp = make_float3(Pv[pn], Pv[ld + pn], Pv[2 * ld + pn]);
    const float w = cv.w[pn];
    const int g = node_group ? node_group[pn] : 0;
    const SurfaceView sv = svs[g];
    int cnt = 0;
    float3 acc = make_float3(0.0f, 0.0f, 0.0f);
    if (node && w != 0.0f && sv.n_tris > 0) {
        const int4 G = groups[g];  // node_off, nx, ny
        const int id = order[pn], loc = id - G.x, nx = G.y, ny = G.z;
        const int row = loc / nx, col = loc - row * nx;
        // cloth-edge neighbours in the order (0,+1) (0,-1) (+1,0) (-1,0) (+1,+1) (-1,-1);
        // absent ones have ok = false
        const int dr[6] = {0, 0, 1, -1, 1, -1}, dc[6] = {1, -1, 0, 0, 1, -1};
        float3 q[6];
        bool ok[6];
        int nid[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const int r2 = row + dr[k], c2 = col + dc[k];
            ok[k] = r2 >= 0 && c2 >= 0 && r2 < ny && c2 < nx;
            nid[k] = id + dr[k] * nx + dc[k];
            const int sk = ok[k] ? slot[nid[k]] : pn;
            q[k] = make_float3(P[sk], P[ld + sk], P[2 * ld + sk]);
        }
        const float3 x0 = make_float3(xs[pn], xs[ld + pn], xs[2 * ld + pn]);
        // query box: path and neighbours (every cloth triangle at i is spanned by them)
        float3 lo = make_float3(fminf(x0.x, xp.x), fminf(x0.y, xp.y), fminf(x0.z, xp.z));
        float3 hi = make_float3(fmaxf(x0.x, xp.x), fmaxf(x0.y, xp.y), fmaxf(x0.z, xp.z));
#pragma unroll
        for (int k = 0; k < 6; ++k)
            if (ok[k]) {
                lo = make_float3(fminf(lo.x, q[k].x), fminf(lo.y, q[k].y), fminf(lo.z, q[k].z));
                hi = make_float3(fmaxf(hi.x, q[k].x), fmaxf(hi.y, q[k].y), fmaxf(hi.z, q[k].z));
            }
        // cloth triangles at i (the split of the quads around it), vertices in (a, b, c) /
        // (a, c, d) order; neighbour index 6 stands for i itself
        //   quad (r-1, c-1): (ul, l, i), (ul, i, u)   quad (r-1, c): (u, i, r)
        //   quad (r, c-1):   (l, d, i)                quad (r, c):   (i, d, dr), (i, dr, r)
        // with r = 0, l = 1, d = 2, u = 3, dr = 4, ul = 5
        const int T0[6] = {5, 5, 3, 1, 6, 6}, T1[6] = {1, 6, 6, 2, 2, 4}, T2[6] = {6, 3, 0, 6, 4, 0};
        bool tok[6];
        tok[0] = ok[5] && ok[1] && ok[3];
        tok[1] = tok[0];
        tok[2] = ok[3] && ok[0];
        tok[3] = ok[1] && ok[2];
        tok[4] = ok[2] && ok[4] && ok[0];
        tok[5] = tok[4];
        auto vert = [&](int k) { return k == 6 ? xp : q[k]; };
        // cell range of the query box, clamped to the grid (boxes outside the grid hold no
        // triangles)
        const float fl0 = cell_coord_f(lo.x, sv.org[0], sv.inv_cell), fh0 = cell_coord_f(hi.x, sv.org[0], sv.inv_cell);
        const float fl1 = cell_coord_f(lo.y, sv.org[1], sv.inv_cell), fh1 = cell_coord_f(hi.y, sv.org[1], sv.inv_cell);
        const float fl2 = cell_coord_f(lo.z, sv.org[2], sv.inv_cell), fh2 = cell_coord_f(hi.z, sv.org[2], sv.inv_cell);
        const bool inside = fh0 >= 0.0f && fh1 >= 0.0f && fh2 >= 0.0f &&
                            fl0 <= (float)(sv.dim[0] - 1) && fl1 <= (float)(sv.dim[1] - 1) &&
                            fl2 <= (float)(sv.dim[2] - 1);
        if (inside) {
            const int q0x = cell_axis(lo.x, sv.org[0], sv.inv_cell, sv.dim[0]);
            const int q0y = cell_axis(lo.y, sv.org[1], sv.inv_cell, sv.dim[1]);
            const int q0z = cell_axis(lo.z, sv.org[2], sv.inv_cell, sv.dim[2]);
            const int q1x = cell_axis(hi.x, sv.org[0], sv.inv_cell, sv.dim[0]);
            const int q1y = cell_axis(hi.y, sv.org[1], sv.inv_cell, sv.dim[1]);
            const int q1z = cell_axis(hi.z, sv.org[2], sv.inv_cell, sv.dim[2]);
            const float th = sv.thickness;
            // the grid's boxes are the triangles' grown by th: shrink them to the triangle
            // plus the margin
            const float shrink = fmaxf(th - fmaxf(th * kMtBoxMargin, 1e-6f), 0.0f);
            auto own_box = [&](float4& blo, float4& bhi) {
                blo = make_float4(blo.x + shrink, blo.y + shrink, blo.z + shrink, blo.w);
                bhi = make_float4(bhi.x - shrink, bhi.y - shrink, bhi.z - shrink, bhi.w);
            };
            // one candidate: does any of the node's segments cross triangle t, or an edge of t
            // cross one of the node's cloth triangles?
            auto test = [&](uint32_t t, const float4& blo, const float4& bhi, const float4& a0,
                            const float4& a1, const float4& a2) {
                const float3 V0 = f3(a0), V1 = f3(a1), V2 = f3(a2);
                // cheap rejections before each segment test: a crossing needs the segment's
                // ends on both sides of (or on) the triangle's plane, and the segment's box
                // to meet the triangle's box
                const float3 Nt = cross3(sub3(V1, V0), sub3(V2, V0));
                const float sp_ = dot3(sub3(xp, V0), Nt);
                bool hit = false;
                if (straddles(dot3(sub3(x0, V0), Nt), sp_) && seg_meets_box(x0, xp, blo, bhi))
                    hit = mt_cross(x0, xp, V0, V1, V2);  // (C)
#pragma unroll
                for (int k = 0; k < 6; ++k)  // (A)
                    if (!hit && ok[k] && straddles(sp_, dot3(sub3(q[k], V0), Nt)) &&
                        seg_meets_box(xp, q[k], blo, bhi))
                        hit = id < nid[k] ? mt_cross(xp, q[k], V0, V1, V2)
                                          : mt_cross(q[k], xp, V0, V1, V2);
                const float3 Vs[3] = {V0, V1, V2};
                const int vid[3] = {__float_as_int(a0.w), __float_as_int(a1.w),
                                    __float_as_int(a2.w)};
#pragma unroll
                for (int k = 0; k < 6; ++k) {  // (B)
                    if (hit || !tok[k]) continue;
                    const float3 P0 = vert(T0[k]), P1 = vert(T1[k]), P2 = vert(T2[k]);
                    if (!tri_meets_box(P0, P1, P2, blo, bhi)) continue;
                    const float3 Nc = cross3(sub3(P1, P0), sub3(P2, P0));
                    float sv3[3];
#pragma unroll
                    for (int z = 0; z < 3; ++z) sv3[z] = dot3(sub3(Vs[z], P0), Nc);
#pragma unroll
                    for (int z = 0; z < 3; ++z) {
                        const int z1 = z == 2 ? 0 : z + 1;
                        if (hit || !straddles(sv3[z], sv3[z1])) continue;
                        const bool fwd = vid[z] < vid[z1];
                        const float3 S = fwd ? Vs[z] : Vs[z1], E = fwd ? Vs[z1] : Vs[z];
                        hit = mt_cross(S, E, P0, P1, P2);
                    }
                }
                if (hit) {
                    if (DEBUG) {
                        if (cnt < cap) ids[(size_t)p * cap + cnt] = (int)t;
                    } else {
                        const float4 g0 = ldg4(sv.geo, 3 * (size_t)t),
                                     g1 = ldg4(sv.geo, 3 * (size_t)t + 1),
                                     g2 = ldg4(sv.geo, 3 * (size_t)t + 2);
                        const float3 n = make_float3(g0.w, g1.w, g2.w);
                        const float s = dot3(sub3(xp, f3(g0)), n);
                        const float push = th - s;
                        acc.x += push * n.x;
                        acc.y += push * n.y;
                        acc.z += push * n.z;
                    }
                    ++cnt;
                }
            };
            // Listing and testing alternate in one loop so the tests are compiled once: a
            // lane lists candidates from its query cells, kMtRefRound references per round of
            // loads (the padding after the last reference keeps a round in bounds), and the
            // lanes of the wavefront test their listed candidates together, in listing order,
            // each triangle's box and vertices loaded one candidate ahead.  A triangle whose
            // box meets the query box is listed in the first query cell that lists it, so
            // each candidate is listed once.  A lane takes the query cells whose ordinal (x
            // fastest, then y, then z) is its share modulo LANES.
            int cx = q0x, cy = q0y, cz = q0z, ci = 0;
            uint32_t r = 0, e = 0;
            if (share == 0) {
                r = gmem(sv.cell_start)[(cz * sv.dim[1] + cy) * sv.dim[0] + cx];
                e = gmem(sv.cell_start)[(cz * sv.dim[1] + cy) * sv.dim[0] + cx + 1];
            }
            bool done = false;
            int nl = 0;
            for (;;) {
                while (!done && r >= e) {  // the next query cell (of this lane's share)
                    if (++cx > q1x) {
                        cx = q0x;
                        if (++cy > q1y) {
                            cy = q0y;
                            if (++cz > q1z) done = true;
                        }
                    }
                    ++ci;
                    if (!done && ci % LANES == share) {
                        const int cell = (cz * sv.dim[1] + cy) * sv.dim[0] + cx;
                        r = gmem(sv.cell_start)[cell];
                        e = gmem(sv.cell_start)[cell + 1];
                    }
                }
                // the lanes test their lists together (the tests are long): when any lane's
                // list could overflow in the next round, and once every lane is done
                const bool all_done = __all(done);
                if (all_done || __any(nl > kMtSlots - kMtRefRound)) {
                    uint32_t t = nl > 0 ? list[0] : 0u;
                    float4 blo = ldg4(sv.box_lo, t), bhi = ldg4(sv.box_hi, t);
                    own_box(blo, bhi);
                    float4 v0 = ldg4(sv.tri_v, 3 * (size_t)t), v1 = ldg4(sv.tri_v, 3 * (size_t)t + 1),
                           v2 = ldg4(sv.tri_v, 3 * (size_t)t + 2);
                    for (int h = 0; h < nl; ++h) {
                        const uint32_t tc = t;
                        const float4 clo = blo, chi = bhi, c0 = v0, c1 = v1, c2 = v2;
                        t = list[min(h + 1, nl - 1) * 64];
                        blo = ldg4(sv.box_lo, t);
                        bhi = ldg4(sv.box_hi, t);
                        own_box(blo, bhi);
                        v0 = ldg4(sv.tri_v, 3 * (size_t)t);
                        v1 = ldg4(sv.tri_v, 3 * (size_t)t + 1);
                        v2 = ldg4(sv.tri_v, 3 * (size_t)t + 2);
                        test(tc, clo, chi, c0, c1, c2);
                    }
                    nl = 0;
                }
                if (all_done) break;
                if (done) continue;  // waits for the wavefront's other lanes
                float4 blo[kMtRefRound], bhi[kMtRefRound];
#pragma unroll
                for (int k = 0; k < kMtRefRound; ++k) {
                    blo[k] = ldg4(sv.ref_lo, r + k);
                    bhi[k] = ldg4(sv.ref_hi, r + k);
                }
#pragma unroll
                for (int k = 0; k < kMtRefRound; ++k) {
                    // (the first-cell test below takes the grid's box, which chose the cells)
                    float4 olo = blo[k], ohi = bhi[k];
                    own_box(olo, ohi);
                    const bool meets = r + k < e && !(ohi.x < lo.x || olo.x > hi.x ||
                                                      ohi.y < lo.y || olo.y > hi.y ||
                                                      ohi.z < lo.z || olo.z > hi.z);
                    const bool first =
                        max(cell_axis(blo[k].x, sv.org[0], sv.inv_cell, sv.dim[0]), q0x) == cx &&
                        max(cell_axis(blo[k].y, sv.org[1], sv.inv_cell, sv.dim[1]), q0y) == cy &&
                        max(cell_axis(blo[k].z, sv.org[2], sv.inv_cell, sv.dim[2]), q0z) == cz;
                    list[nl * 64] = (uint32_t)__float_as_int(blo[k].w);
                    nl += meets && first ? 1 : 0;
                }
                r += kMtRefRound;
            }
        }
    }
    if (DEBUG) {
        counts[p] = cnt;
        return;
    }
    if constexpr (SPLIT) {
        // the other lanes' sums and counts, added to the first's in lane order
        if (share > 0) part[share - 1][pair] = make_float4(acc.x, acc.y, acc.z, __int_as_float(cnt));
        __syncthreads();
        if (share > 0 || !node) return;
#pragma unroll
        for (int j = 0; j < LANES - 1; ++j) {
            const float4 o = part[j][pair];
            acc.x += o.x;
            acc.y += o.y;
            acc.z += o.z;
            cnt += __float_as_int(o.w);
        }
    }
    if (cnt > 0) {
        const float inv = 1.0f / (float)cnt;
        xp.x += acc.x * inv;
        xp.y += acc.y * inv;
        xp.z += acc.z * inv;
        vp.x = -sp.restitution * vp.x;
        vp.y = -sp.restitution * vp.y;
        vp.z = -sp.restitution * vp.z;
    }
    xd[p] = xp.x;
    xd[ld + p] = xp.y;
    xd[2 * ld + p] = xp.z;
    vd[p] = vp.x;
    vd[ld + p] = vp.y;
    vd[2 * ld + p] = vp.z;
    if (sp.check_nan) {
        const float sum = xp.x + xp.y + xp.z + vp.x + vp.y + vp.z;
        if (!__builtin_isfinite(sum)) atomicOr(sp.nan_flag, 1);
    }
}

}  // namespace

hipError_t launch_mt_substep(const ClothView& cv, const StepParams& sp, const MtTopology& tp,
                             const SurfaceView* svs, const float* xs, const float* vs, float* P,
                             float* xd, float* vd, int block, hipStream_t st) {
    if (cv.n <= 0) return hipSuccess;
    // prediction without collision into P, then the contact search and response
    hipError_t e = launch_substep(cv, 0, sp, xs, vs, P, P + 3 * (size_t)cv.ld, block, st, svs);
    if (e != hipSuccess) return e;
    constexpr int per = mt_nodes_per_block<kMtLanes>();
    k_mt_collide<false, kMtLanes><<<(cv.n + per - 1) / per, 256, 0, st>>>(
        cv, sp, tp.order, tp.slot, tp.node_group, tp.groups, svs, xs, P, xd, vd, nullptr, nullptr,
        0);
    return hipGetLastError();
}

hipError_t launch_mt_debug_contacts(const ClothView& cv, const StepParams& sp,
                                    const MtTopology& tp, const SurfaceView* svs, const float* xs,
                                    const float* vs, float* P, int* counts, int* ids, int cap,
                                    hipStream_t st) {
    if (cv.n <= 0) return hipSuccess;
    hipError_t e = launch_substep(cv, 0, sp, xs, vs, P, P + 3 * (size_t)cv.ld, 256, st, svs);
    if (e != hipSuccess) return e;
    constexpr int per = mt_nodes_per_block<1>();
    k_mt_collide<true, 1><<<(cv.n + per - 1) / per, 256, 0, st>>>(
        cv, sp, tp.order, tp.slot, tp.node_group, tp.groups, svs, xs, P, nullptr, nullptr, counts,
        ids, cap);
    return hipGetLastError();
}

}  // namespace cloth
