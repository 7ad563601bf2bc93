// Device helpers shared by the HIP kernels: grid cell mapping, inflated-box test, spring
// force of one incidence, and point-triangle closest-point distance.
#pragma once

#include <hip/hip_runtime.h>

#include "cloth_internal.h"

namespace cloth {

// Loads through these pointers are global-memory loads: the flat form the compiler uses for
// pointers it cannot place (fields of structures read from device memory) also counts
// against the LDS wait counter, which serialises global loads with LDS traffic.
template <class T>
using gptr = const __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ gptr<T> gmem(const T* p) {
    return (gptr<T>)p;
}
typedef float f32x4 __attribute__((ext_vector_type(4)));
// Element i of a float4 array, as one global 16-byte load.
__device__ __forceinline__ float4 ldg4(const float4* p, size_t i) {
    const f32x4 v = gmem(reinterpret_cast<const f32x4*>(p))[i];
    return make_float4(v.x, v.y, v.z, v.w);
}

// Logical workgroup of this workgroup.  The hardware deals workgroup b to XCD b mod 8, and
// each XCD has its own L2.  xcd_runs = 0 keeps that order; 1 gives each XCD one contiguous
// run of the logical workgroups; k >= 2 deals chunks of k consecutive logical workgroups to
// the XCDs in turn (XCD x holds chunks x, x + 8, ...), so an XCD's nodes are spatially
// coherent pieces spread over the whole cloth.  For k >= 2 the grid is padded to a multiple
// of 8k (xcd_grid) and a padding workgroup gets n_logical, i.e. no valid node.
__device__ __forceinline__ int xcd_block(int xcd_runs, int n_logical) {
    const int b = blockIdx.x, x8 = b & 7, j = b >> 3;
    if (xcd_runs == 0) return b;
    if (xcd_runs == 1) {
        const int q8 = n_logical >> 3, rem = n_logical & 7;
        return x8 * q8 + (x8 < rem ? x8 : rem) + j;
    }
    const int blk = ((j / xcd_runs) * 8 + x8) * xcd_runs + j % xcd_runs;
    return blk < n_logical ? blk : n_logical;
}

// Unclamped grid coordinate of one axis, floor((p - org) * inv_cell) in FP32.  Monotone
// non-decreasing in p (each FP32 operation rounds to nearest and floor is monotone), so a
// triangle registered in the cells cell(lo)..cell(hi) of its inflated box is found from
// any point inside the box.  No contraction: build and query must agree bit for bit.
__device__ __forceinline__ float cell_coord_raw(float p, float org, float inv_cell) {
#pragma clang fp contract(off)
    return (p - org) * inv_cell;
}
__device__ __forceinline__ float cell_coord_f(float p, float org, float inv_cell) {
    return floorf(cell_coord_raw(p, org, inv_cell));
}

// Coded box test.  On each axis, g = (p - org) * inv_cell as computed above is monotone in
// p, so g(p) < g(lo) implies p < lo and g(p) > g(lo) implies p > lo.  Within the cell c the
// bucket Q(p) = floor((g(p) - c) * 2^15) is computed exactly (the difference and the
// scaling are exact for g in [c, c + 1)), so comparing buckets decides lo <= p <= hi except
// when p shares a bucket with lo or hi.  A reference stores per axis the 32-bit word
// (Q(lo) + 1) | (0xffff - Q(hi)) << 16, with Q(lo) + 1 = 0 when lo lies before the cell and
// Q(hi) = 2^15 when hi lies beyond it; the point uses Q(p) | (0xfffe - Q(p)) << 16.  The
// saturating 16-bit differences word - point are 0 when the axis is certainly inside, 1
// when p shares a bucket with lo or hi and at least 2 when it is certainly outside, so the
// maximum over the six halves is 0 for a box hit, 1 for "decide with the exact box" and
// >= 2 for a miss.
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
constexpr int kCodeBits = 15;
__device__ __forceinline__ uint32_t point_code(float g, float c) {
#pragma clang fp contract(off)
    const int q = (int)floorf((g - c) * (float)(1 << kCodeBits));  // 0 .. 2^15 - 1
    return (uint32_t)q | ((uint32_t)(0xfffe - q) << 16);
}
__device__ __forceinline__ uint32_t box_code(const uint4& w, uint32_t cx, uint32_t cy,
                                             uint32_t cz) {
    const u16x2 tx = __builtin_elementwise_sub_sat(__builtin_bit_cast(u16x2, w.x),
                                                   __builtin_bit_cast(u16x2, cx));
    const u16x2 ty = __builtin_elementwise_sub_sat(__builtin_bit_cast(u16x2, w.y),
                                                   __builtin_bit_cast(u16x2, cy));
    const u16x2 tz = __builtin_elementwise_sub_sat(__builtin_bit_cast(u16x2, w.z),
                                                   __builtin_bit_cast(u16x2, cz));
    const u16x2 m = __builtin_elementwise_max(__builtin_elementwise_max(tx, ty), tz);
    return (uint32_t)(m.x > m.y ? m.x : m.y);
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
// Element i of a uint4 array, as one global 16-byte load.
__device__ __forceinline__ uint4 ldgu4(const uint4* p, size_t i) {
    const u32x4 v = gmem(reinterpret_cast<const u32x4*>(p))[i];
    return make_uint4(v.x, v.y, v.z, v.w);
}
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
// Element i of a uint2 array, as one global 8-byte load.
__device__ __forceinline__ uint2 ldgu2(const uint2* p, size_t i) {
    const u32x2 v = gmem(reinterpret_cast<const u32x2*>(p))[i];
    return make_uint2(v.x, v.y);
}

__device__ __forceinline__ int cell_axis(float p, float org, float inv_cell, int dim) {
    float f = cell_coord_f(p, org, inv_cell);
    f = fminf(fmaxf(f, 0.0f), (float)(dim - 1));  // NaN -> 0
    return (int)f;
}

// Cell of a query point, or -1 when the point lies outside the grid.  The grid's origin is
// at or below every inflated box's low corner and its dims are chosen so every high corner
// maps to at most dim - 1, so by monotonicity no box contains a point whose coordinate maps
// outside [0, dim - 1].  NaN maps to -1.
__device__ __forceinline__ int cell_of(const SurfaceView& sv, float px, float py, float pz) {
    const float fx = cell_coord_f(px, sv.org[0], sv.inv_cell);
    const float fy = cell_coord_f(py, sv.org[1], sv.inv_cell);
    const float fz = cell_coord_f(pz, sv.org[2], sv.inv_cell);
    if (!(fx >= 0.0f && fx <= (float)(sv.dim[0] - 1) && fy >= 0.0f &&
          fy <= (float)(sv.dim[1] - 1) && fz >= 0.0f && fz <= (float)(sv.dim[2] - 1)))
        return -1;
    return ((int)fz * sv.dim[1] + (int)fy) * sv.dim[0] + (int)fx;
}

// Inclusive inflated-box test (the broad-phase predicate).
__device__ __forceinline__ bool in_box(const float4& lo, const float4& hi, float px, float py,
                                       float pz) {
    return lo.x <= px && px <= hi.x && lo.y <= py && py <= hi.y && lo.z <= pz && pz <= hi.z;
}

// Force on node i from one spring to neighbour j (Alg. 1 with i as indexA):
//   d = x_j - x_i, l = |d|, f = (k (l - L0) + c (v_j - v_i).d / l) d / l = s d.
// 1/l comes from the hardware reciprocal square root (about 1 ulp).  spring_coeff gives s,
// spring_accumulate adds s d to the node's sum; every force kernel sums its incidences with
// these two, in incidence order, so all of them produce the same bits.
__device__ __forceinline__ float spring_coeff(float dx, float dy, float dz, float dvx, float dvy,
                                              float dvz, float k, float c, float L0) {
    float l2 = dx * dx + dy * dy + dz * dz;
    float il = __builtin_amdgcn_rsqf(l2);
    float l = l2 * il;
    float phi = k * (l - L0) + c * (dvx * dx + dvy * dy + dvz * dz) * il;
    return phi * il;
}
__device__ __forceinline__ void spring_accumulate(float s, float dx, float dy, float dz, float& fx,
                                                  float& fy, float& fz) {
    fx += s * dx;
    fy += s * dy;
    fz += s * dz;
}
__device__ __forceinline__ void spring_force(float dx, float dy, float dz, float dvx, float dvy,
                                             float dvz, float k, float c, float L0, float& fx,
                                             float& fy, float& fz) {
    spring_accumulate(spring_coeff(dx, dy, dz, dvx, dvy, dvz, k, c, L0), dx, dy, dz, fx, fy, fz);
}

// a1 gather of one node over a sliced-CSR incidence list in global memory, up to twelve
// incidences per round (a grid cloth's interior degree): all their records, then all their
// springs' parameters and neighbours' states, are loaded back to back (indices clamped to
// the list, so no load depends on a branch), and the forces are then summed in incidence
// order, which keeps the sum identical to a one-by-one loop.
__device__ __forceinline__ void gather_global(const ClothView& cv, const float* __restrict__ xs,
                                              const float* __restrict__ vs, int i, float xi,
                                              float yi, float zi, float vxi, float vyi,
                                              float vzi, float& fx, float& fy, float& fz) {
    constexpr int R = 12;
    const int ld = cv.ld;
    const int deg = cv.deg[i];
    const int base = cv.slice_ptr[i >> 6] + (i & 63);
    const gptr<float> X = gmem(xs), V = gmem(vs);
    for (int r0 = 0; r0 < deg; r0 += R) {
        uint2 rec[R];
#pragma unroll
        for (int q = 0; q < R; ++q) rec[q] = ldgu2(cv.inc2, (size_t)(base + min(r0 + q, deg - 1) * 64));
        float4 e[R];  // (k, c, rest length, 0)
        float nx[R], ny[R], nz[R], mx[R], my[R], mz[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            e[q] = ldg4(cv.ptab, rec[q].y);
            const int j = (int)rec[q].x;
            nx[q] = X[j];
            ny[q] = X[ld + j];
            nz[q] = X[2 * ld + j];
            mx[q] = V[j];
            my[q] = V[ld + j];
            mz[q] = V[2 * ld + j];
        }
#pragma unroll
        for (int q = 0; q < R; ++q)
            if (r0 + q < deg)
                spring_force(nx[q] - xi, ny[q] - yi, nz[q] - zi, mx[q] - vxi, my[q] - vyi,
                             mz[q] - vzi, e[q].x, e[q].y, e[q].z, fx, fy, fz);
    }
}

// Squared distance from p to triangle (A, A+e1, A+e2); ap = p - A, s = ap . n (signed plane
// distance along the unit normal n).  The closest point of the triangle is p's projection on
// its plane when that projection lies inside the triangle (distance |s|), else the closest
// point of one of its three edges.  Branch- and division-free: an edge e from P is reached
// at the clamped parameter t = clamp((p - P).e / |e|^2, 0, 1) (the quotient through the
// hardware reciprocal) at squared distance |p - P - t e|^2, formed from the vector so that
// its rounding error scales with the distance, not with |p - P|.  The inside test uses the
// barycentric numerators of the projection over the Gram matrix of (e1, e2); on the
// boundary the face and edge distances coincide, so rounding in that test moves the result
// by no more than rounding in the distances does.
__device__ __forceinline__ float edge_dist2(float px, float py, float pz, float ex, float ey,
                                            float ez, float pe, float ee) {
    const float t = fminf(fmaxf(pe * __builtin_amdgcn_rcpf(ee), 0.0f), 1.0f);
    const float qx = px - t * ex, qy = py - t * ey, qz = pz - t * ez;
    return qx * qx + qy * qy + qz * qz;
}

__device__ __forceinline__ float point_tri_dist2(float apx, float apy, float apz, float e1x,
                                                 float e1y, float e1z, float e2x, float e2y,
                                                 float e2z, float s) {
    const float d1 = e1x * apx + e1y * apy + e1z * apz;
    const float d2 = e2x * apx + e2y * apy + e2z * apz;
    const float g11 = e1x * e1x + e1y * e1y + e1z * e1z;
    const float g22 = e2x * e2x + e2y * e2y + e2z * e2z;
    const float g12 = e1x * e2x + e1y * e2y + e1z * e2z;
    const float dab = edge_dist2(apx, apy, apz, e1x, e1y, e1z, d1, g11);
    const float dac = edge_dist2(apx, apy, apz, e2x, e2y, e2z, d2, g22);
    const float e3x = e2x - e1x, e3y = e2y - e1y, e3z = e2z - e1z;  // C - B
    const float bpx = apx - e1x, bpy = apy - e1y, bpz = apz - e1z;  // p - B
    const float d3 = e3x * bpx + e3y * bpy + e3z * bpz;
    const float g33 = e3x * e3x + e3y * e3y + e3z * e3z;
    const float dbc = edge_dist2(bpx, bpy, bpz, e3x, e3y, e3z, d3, g33);
    // projection = A + (u e1 + v e2) / det with det = |e1 x e2|^2 > 0
    const float u = g22 * d1 - g12 * d2;
    const float v = g11 * d2 - g12 * d1;
    const float det = g11 * g22 - g12 * g12;
    const bool inside = (u >= 0.0f) & (v >= 0.0f) & (u + v <= det);
    // every edge distance is >= s^2, so the minimum below is s^2 inside and the nearest
    // edge's distance outside; written this way no lane skips the edge terms
    return fminf(inside ? s * s : __builtin_inff(), fminf(fminf(dab, dac), dbc));
}

// External force of the node in internal slot `slot`, added to its spring-force sum.
__device__ __forceinline__ void add_external(const StepParams& sp, int slot, float& fx, float& fy,
                                             float& fz) {
    if (sp.fext) {
        fx += sp.fext[slot];
        fy += sp.fext[sp.fext_ld + slot];
        fz += sp.fext[2 * sp.fext_ld + slot];
    }
}

// a2: semi-implicit Euler for one node; pinned nodes (w = 0) keep x and get v* = 0.
__device__ __forceinline__ void integrate(float w, float h, const float g[3], float xi, float yi,
                                          float zi, float vxi, float vyi, float vzi, float fx,
                                          float fy, float fz, float& px, float& py, float& pz,
                                          float& qx, float& qy, float& qz) {
    px = xi;
    py = yi;
    pz = zi;
    qx = qy = qz = 0.0f;
    if (w != 0.0f) {
        qx = vxi + h * (w * fx + g[0]);
        qy = vyi + h * (w * fy + g[1]);
        qz = vzi + h * (w * fz + g[2]);
        px = xi + h * qx;
        py = yi + h * qy;
        pz = zi + h * qz;
    }
}

// Narrow phase against one broad-phase candidate whose packed geometry (A, n.x), (B-A, n.y),
// (C-A, n.z) is g0, g1, g2: contact iff the point-triangle distance is < thickness; then
// visit(n, s, t).  Returns 1 for a contact.
// The unit normal n of a candidate's packed geometry (A, n.x), (B-A, n.y), (C-A, n.z), the
// vector a = p - A and the signed plane distance s = a.n (returned).
__device__ __forceinline__ float plane_offset(const float4& g0, const float4& g1,
                                              const float4& g2, float px, float py, float pz,
                                              float4& n, float& ax, float& ay, float& az) {
    n = make_float4(g0.w, g1.w, g2.w, 0.0f);
    ax = px - g0.x;
    ay = py - g0.y;
    az = pz - g0.z;
    return ax * n.x + ay * n.y + az * n.z;
}

template <class Visit>
__device__ __forceinline__ int narrow_visit(const SurfaceView& sv, uint32_t t, const float4& g0,
                                            const float4& g1, const float4& g2, float px,
                                            float py, float pz, Visit&& visit) {
    float4 n;
    float ax, ay, az;
    const float s = plane_offset(g0, g1, g2, px, py, pz, n, ax, ay, az);
    const float d2 = point_tri_dist2(ax, ay, az, g1.x, g1.y, g1.z, g2.x, g2.y, g2.z, s);
    if (d2 < sv.thickness2) {
        visit(n, s, t);
        return 1;
    }
    return 0;
}

// Position (0..63) of the lowest set bit, and that bit cleared.
__device__ __forceinline__ int pop_low(unsigned long long& m) {
    const int k = __builtin_ctzll(m);
    m &= m - 1ULL;
    return k;
}

// Narrow phase of up to four box hits whose triangle ids are t[0..n) (ascending): their
// geometry loads are issued together (ids past n repeat the last one and are not visited).
template <class Visit>
__device__ __forceinline__ int narrow4(const SurfaceView& sv, uint32_t t0, uint32_t t1, uint32_t t2,
                                       uint32_t t3, int n, float px, float py, float pz,
                                       Visit&& visit) {
    const uint32_t t[4] = {t0, t1, t2, t3};
    float4 g[4][3];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        g[q][0] = ldg4(sv.geo, 3 * (size_t)t[q]);
        g[q][1] = ldg4(sv.geo, 3 * (size_t)t[q] + 1);
        g[q][2] = ldg4(sv.geo, 3 * (size_t)t[q] + 2);
    }
    int cnt = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (q < n) cnt += narrow_visit(sv, t[q], g[q][0], g[q][1], g[q][2], px, py, pz, visit);
    return cnt;
}

// Visits the box hits recorded in `mask` (bit k = entry k of a run of references, ascending
// triangle id), four per round of geometry loads; id(k) gives entry k's triangle id.
template <class Id, class Visit>
__device__ __forceinline__ int narrow_mask(const SurfaceView& sv, unsigned long long mask, Id&& id,
                                           float px, float py, float pz, Visit&& visit) {
    int cnt = 0;
    while (mask) {
        const int n = min(__popcll(mask), 4);
        const int k0 = pop_low(mask);
        const int k1 = n > 1 ? pop_low(mask) : k0;
        const int k2 = n > 2 ? pop_low(mask) : k1;
        const int k3 = n > 3 ? pop_low(mask) : k2;
        cnt += narrow4(sv, id(k0), id(k1), id(k2), id(k3), n, px, py, pz, visit);
    }
    return cnt;
}

// a3 + a4 contact search over the references [b, e) of the grid cell of a node at predicted
// position p: candidates are the listed triangles whose inflated box holds p (ascending
// id); a candidate is a contact iff the point-triangle distance is < thickness, and
// visit(n, s, t) is then called with the triangle's unit normal n, the signed plane distance
// s = (p - A).n and the triangle id t.  Reference boxes are loaded RR (<= kRefRound) at a time
// (the arrays carry kRefRound entries of padding, so the loads need no bounds test).  Returns
// the contact count.  NARROW = false stops after the broad phase: every candidate is visited (n
// and s are zero) and counted.
template <bool NARROW = true, int RR = kRefRound, class Visit>
__device__ __forceinline__ int visit_range(const SurfaceView& sv, uint32_t b, uint32_t e,
                                           float px, float py, float pz, Visit&& visit) {
    int cnt = 0;
    for (uint32_t r = b; r < e; r += RR) {
        float4 lo[RR], hi[RR];
#pragma unroll
        for (int q = 0; q < RR; ++q) {
            lo[q] = ldg4(sv.ref_lo, r + q);
            hi[q] = ldg4(sv.ref_hi, r + q);
        }
        unsigned long long mask = 0;
#pragma unroll
        for (int q = 0; q < RR; ++q)
            if (r + q < e && in_box(lo[q], hi[q], px, py, pz)) mask |= 1ULL << q;
        // a hit's triangle id is re-read from the box just loaded (a cache hit): selecting it
        // from the registers above would make the compiler spill them to scratch
        auto id = [&](int k) {
            return (uint32_t)gmem(reinterpret_cast<const int*>(sv.ref_lo))[4 * (size_t)(r + k) + 3];
        };
        if constexpr (NARROW) {
            cnt += narrow_mask(sv, mask, id, px, py, pz, visit);
        } else {
            while (mask) {
                visit(make_float4(0.0f, 0.0f, 0.0f, 0.0f), 0.0f, id(pop_low(mask)));
                ++cnt;
            }
        }
    }
    return cnt;
}

// visit_range over the whole cell of p (no candidates outside the grid).
template <bool NARROW = true, class Visit>
__device__ __forceinline__ int contacts_visit(const SurfaceView& sv, float px, float py, float pz,
                                              Visit&& visit) {
    const int cell = cell_of(sv, px, py, pz);
    if (cell < 0) return 0;
    const gptr<uint32_t> cs = gmem(sv.cell_start);
    return visit_range<NARROW>(sv, cs[cell], cs[cell + 1], px, py, pz, visit);
}

// The sum that the averaged response divides by the contact count: (th - s) n over the
// contacts, in the order they are visited (a visitor for the contact searches).
struct PushSum {
    float th;
    float x = 0.0f, y = 0.0f, z = 0.0f;
    __device__ explicit PushSum(float thickness) : th(thickness) {}
    __device__ __forceinline__ void operator()(const float4& n, float s, uint32_t) {
        const float push = th - s;
        x += push * n.x;
        y += push * n.y;
        z += push * n.z;
    }
};

// Response of Alg. 2 with the averaged direction: with at least one contact, p moves by the
// mean of (th - s_t) n_t over the contacts and q becomes -restitution q.
__device__ __forceinline__ void respond(int cnt, float sx, float sy, float sz, float restitution,
                                        float& px, float& py, float& pz, float& qx, float& qy,
                                        float& qz) {
    if (cnt > 0) {
        const float inv = 1.0f / (float)cnt;
        px += sx * inv;
        py += sy * inv;
        pz += sz * inv;
        qx = -restitution * qx;
        qy = -restitution * qy;
        qz = -restitution * qz;
    }
}

__device__ __forceinline__ int collide(const SurfaceView& sv, float restitution, float& px,
                                       float& py, float& pz, float& qx, float& qy, float& qz) {
    PushSum sum(sv.thickness);
    const int cnt = contacts_visit(sv, px, py, pz, sum);
    respond(cnt, sum.x, sum.y, sum.z, restitution, px, py, pz, qx, qy, qz);
    return cnt;
}

// The box hits among the references [b, e) of p's grid cell (cx, cy, cz: p's point codes in
// that cell, see point_code), appended to this lane's list in LDS in reference order
// (ascending triangle id): the coded reference records are tested RR (<= kRefRound) per
// round of loads, and a hit's triangle id goes to list[k * 64] (k < slots), plus a scratch
// entry k = slots: every reference is written at the next free entry, or at the scratch entry
// once the list is full, and only a hit advances the count.  A hit whose coded test was
// undecided carries bit 31 and is decided with the exact box before its narrow test.
// Returns the number of hits, which may exceed slots (then the list holds the first slots).
template <int RR = kRefRound>
__device__ __forceinline__ int list_box_hits(const SurfaceView& sv, uint32_t* list, int slots,
                                             uint32_t cx, uint32_t cy, uint32_t cz, uint32_t b,
                                             uint32_t e) {
    int nh = 0;
    // a round's entries load from one address at fixed offsets
    auto load = [&](uint4 (&w)[RR], uint32_t r) {
        const uint4* rq = sv.ref_q + r;
#pragma unroll
        for (int q = 0; q < RR; ++q) w[q] = ldgu4(rq, q);
    };
    auto test = [&](const uint4 (&w)[RR], uint32_t r) {
#pragma unroll
        for (int q = 0; q < RR; ++q) {
            const uint32_t m = box_code(w[q], cx, cy, cz);
            list[min(nh, slots) * 64] = w[q].w | (m << 31);
            nh += (r + q < e && m <= 1u) ? 1 : 0;
        }
    };
    // Two rounds in flight: the next round's loads are issued before this round is tested.
    // The loop body has no branch, so the loads stay ahead of the tests and the compiler
    // counts them exactly: every load is unconditional (a lane without a further round
    // reloads its current one, which is cached; an empty cell loads at b <= the reference
    // count, which the arrays' padding covers), and a round past the cell's end is tested
    // without effect (its entries fail r + q < e).
    uint4 wa[RR], wb[RR];
    load(wa, b);
    for (uint32_t r = b; r < e; r += 2 * RR) {
        const uint32_t r1 = r + RR, r2 = r1 + RR;
        load(wb, r1 < e ? r1 : r);
        __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the tests
        test(wa, r);
        load(wa, r2 < e ? r2 : r);
        __builtin_amdgcn_sched_barrier(0);
        test(wb, r1);
    }
    return nh;
}

// One round of the listed box hits: entries h0 .. h0 + HR - 1 of a list of nh (1 <= nh <=
// slots) entries.  Their geometry loads are issued together (entries past nh repeat the last
// one and are not visited), undecided entries are settled with the exact box in one branch
// (which the wavefront skips when none of its lanes has one), and on_hit(k, t, g0, g1, g2) is
// called for each remaining entry k in ascending order, with its triangle id t and packed
// geometry.
template <int HR, class OnHit>
__device__ __forceinline__ void hit_round(const SurfaceView& sv, const uint32_t* list, int nh,
                                          int h0, float px, float py, float pz, OnHit&& on_hit) {
    const int n = min(nh - h0, HR);
    uint32_t t[HR];
    float4 g[HR][3];
#pragma unroll
    for (int q = 0; q < HR; ++q) t[q] = list[min(h0 + q, nh - 1) * 64];
#pragma unroll
    for (int q = 0; q < HR; ++q) {
        const size_t id = t[q] & 0x7fffffffu;
        g[q][0] = ldg4(sv.geo, 3 * id);
        g[q][1] = ldg4(sv.geo, 3 * id + 1);
        g[q][2] = ldg4(sv.geo, 3 * id + 2);
    }
    uint32_t live = (1u << n) - 1u, und = 0;
#pragma unroll
    for (int q = 0; q < HR; ++q) und |= (t[q] >> 31) << q;
    und &= live;
    if (und) {
#pragma unroll
        for (int q = 0; q < HR; ++q)
            if ((und >> q) & 1u) {
                const uint32_t id = t[q] & 0x7fffffffu;
                if (!in_box(ldg4(sv.box_lo, id), ldg4(sv.box_hi, id), px, py, pz))
                    live &= ~(1u << q);
            }
    }
    // (a wavefront skips a slot none of its lanes holds, e.g. in its last round)
#pragma unroll
    for (int q = 0; q < HR; ++q)
        if ((live >> q) & 1u) on_hit(h0 + q, t[q] & 0x7fffffffu, g[q][0], g[q][1], g[q][2]);
}

// a3 + a4 contact search with the box hits of the references [b, e) of p's cell collected
// first (list_box_hits), then their geometry loaded HR hits per round (hit_round), so a node
// with many box hits waits for few round trips.  Contacts are visited in ascending triangle
// id, exactly as visit_range visits them (same contacts, same order); a lane with more hits
// than slots runs visit_range instead.  Returns the contact count.  NARROW = false stops
// after the broad phase: every box hit (undecided ones settled with the exact box) is
// visited, with n and s zero, and counted; this is the query the step kernels run, up to the
// narrow test.
template <bool NARROW = true, int RR = kRefRound, int HR = kHitRound, class Visit>
__device__ __forceinline__ int listed_range(const SurfaceView& sv, uint32_t* list, int slots,
                                            uint32_t cx, uint32_t cy, uint32_t cz, uint32_t b,
                                            uint32_t e, float px, float py, float pz,
                                            Visit&& visit) {
    const int nh = list_box_hits<RR>(sv, list, slots, cx, cy, cz, b, e);
    if (nh > slots) return visit_range<NARROW, RR>(sv, b, e, px, py, pz, visit);
    int contacts = 0;
    if constexpr (!NARROW) {
        for (int k = 0; k < nh; ++k) {
            const uint32_t t = list[k * 64];
            const uint32_t id = t & 0x7fffffffu;
            if ((t >> 31) && !in_box(ldg4(sv.box_lo, id), ldg4(sv.box_hi, id), px, py, pz))
                continue;
            visit(make_float4(0.0f, 0.0f, 0.0f, 0.0f), 0.0f, id);
            ++contacts;
        }
    } else {
        for (int h0 = 0; h0 < nh; h0 += HR)
            hit_round<HR>(sv, list, nh, h0, px, py, pz,
                          [&](int, uint32_t t, const float4& g0, const float4& g1,
                              const float4& g2) {
                              contacts += narrow_visit(sv, t, g0, g1, g2, px, py, pz, visit);
                          });
    }
    return contacts;
}

// p's grid cell: its reference range [b, e) and p's point codes in it (point_code); false
// when p's cell coordinate falls outside the grid (no candidates).
__device__ __forceinline__ bool cell_refs(const SurfaceView& sv, float px, float py, float pz,
                                          uint32_t& cx, uint32_t& cy, uint32_t& cz, uint32_t& b,
                                          uint32_t& e) {
    const float gx = cell_coord_raw(px, sv.org[0], sv.inv_cell);
    const float gy = cell_coord_raw(py, sv.org[1], sv.inv_cell);
    const float gz = cell_coord_raw(pz, sv.org[2], sv.inv_cell);
    const float fx = floorf(gx), fy = floorf(gy), fz = floorf(gz);
    // the test of cell_of, on the same values
    if (!(fx >= 0.0f && fx <= (float)(sv.dim[0] - 1) && fy >= 0.0f &&
          fy <= (float)(sv.dim[1] - 1) && fz >= 0.0f && fz <= (float)(sv.dim[2] - 1)))
        return false;
    const int cell = ((int)fz * sv.dim[1] + (int)fy) * sv.dim[0] + (int)fx;
    cx = point_code(gx, fx);
    cy = point_code(gy, fy);
    cz = point_code(gz, fz);
    const gptr<uint32_t> cs = gmem(sv.cell_start);
    b = cs[cell];
    e = cs[cell + 1];
    return true;
}

// listed_range over the whole cell of p (no candidates outside the grid).  Short rounds of
// box hits (HR <= 4) go with short rounds of references as well: fewer registers, for
// collision work spread over many wavefronts.
template <bool NARROW = true, int HR = kHitRound, class Visit>
__device__ __forceinline__ int contacts_listed(const SurfaceView& sv, uint32_t* list, int slots,
                                               float px, float py, float pz, Visit&& visit) {
    constexpr int RR = HR <= 4 ? 4 : kRefRound;
    uint32_t cx, cy, cz, b, e;
    if (!cell_refs(sv, px, py, pz, cx, cy, cz, b, e)) return 0;
    return listed_range<NARROW, RR, HR>(sv, list, slots, cx, cy, cz, b, e, px, py, pz, visit);
}

// collide_listed: contacts_listed with the averaged response (HR box hits per round of
// geometry loads).
template <int HR = kHitRound>
__device__ __forceinline__ int collide_listed(const SurfaceView& sv, uint32_t* list, int slots,
                                              float restitution, float& px, float& py,
                                              float& pz, float& qx, float& qy, float& qz) {
    PushSum sum(sv.thickness);
    const int contacts = contacts_listed<true, HR>(sv, list, slots, px, py, pz, sum);
    respond(contacts, sum.x, sum.y, sum.z, restitution, px, py, pz, qx, qy, qz);
    return contacts;
}

}  // namespace cloth
