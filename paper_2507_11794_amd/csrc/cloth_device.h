// Device helpers shared by the HIP kernels: grid cell mapping, inflated-box test, spring
// force of one incidence, and point-triangle closest-point distance.
#pragma once

#include <hip/hip_runtime.h>

#include "cloth_internal.h"

namespace cloth {

// Unclamped grid coordinate of one axis, floor((p - org) * inv_cell) in FP32.  Monotone
// non-decreasing in p (each FP32 operation rounds to nearest and floor is monotone), so a
// triangle registered in the cells cell(lo)..cell(hi) of its inflated box is found from
// any point inside the box.  No contraction: build and query must agree bit for bit.
__device__ __forceinline__ float cell_coord_f(float p, float org, float inv_cell) {
#pragma clang fp contract(off)
    return floorf((p - org) * inv_cell);
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
//   d = x_j - x_i, l = |d|, f = (k (l - L0) + c (v_j - v_i).d / l) d / l.
// 1/l comes from the hardware reciprocal square root (about 1 ulp).
__device__ __forceinline__ void spring_force(float dx, float dy, float dz, float dvx, float dvy,
                                             float dvz, float k, float c, float L0, float& fx,
                                             float& fy, float& fz) {
    float l2 = dx * dx + dy * dy + dz * dz;
    float il = __builtin_amdgcn_rsqf(l2);
    float l = l2 * il;
    float phi = k * (l - L0) + c * (dvx * dx + dvy * dy + dvz * dz) * il;
    float s = phi * il;
    fx += s * dx;
    fy += s * dy;
    fz += s * dz;
}

// Squared distance from p to triangle (A, A+e1, A+e2) by Voronoi regions (Ericson,
// Real-Time Collision Detection, Sec. 5.1.5).  ap = p - A; s = ap . n (signed plane
// distance along the unit normal n), used for the face region.
__device__ __forceinline__ float point_tri_dist2(float apx, float apy, float apz, float e1x,
                                                 float e1y, float e1z, float e2x, float e2y,
                                                 float e2z, float s) {
    float d1 = e1x * apx + e1y * apy + e1z * apz;
    float d2 = e2x * apx + e2y * apy + e2z * apz;
    if (d1 <= 0.0f && d2 <= 0.0f) return apx * apx + apy * apy + apz * apz;  // vertex A
    float bpx = apx - e1x, bpy = apy - e1y, bpz = apz - e1z;                  // p - B
    float d3 = e1x * bpx + e1y * bpy + e1z * bpz;
    float d4 = e2x * bpx + e2y * bpy + e2z * bpz;
    if (d3 >= 0.0f && d4 <= d3) return bpx * bpx + bpy * bpy + bpz * bpz;  // vertex B
    float vc = d1 * d4 - d3 * d2;
    if (vc <= 0.0f && d1 >= 0.0f && d3 <= 0.0f) {  // edge AB
        float t = d1 / (d1 - d3);
        float qx = apx - t * e1x, qy = apy - t * e1y, qz = apz - t * e1z;
        return qx * qx + qy * qy + qz * qz;
    }
    float cpx = apx - e2x, cpy = apy - e2y, cpz = apz - e2z;  // p - C
    float d5 = e1x * cpx + e1y * cpy + e1z * cpz;
    float d6 = e2x * cpx + e2y * cpy + e2z * cpz;
    if (d6 >= 0.0f && d5 <= d6) return cpx * cpx + cpy * cpy + cpz * cpz;  // vertex C
    float vb = d5 * d2 - d1 * d6;
    if (vb <= 0.0f && d2 >= 0.0f && d6 <= 0.0f) {  // edge AC
        float t = d2 / (d2 - d6);
        float qx = apx - t * e2x, qy = apy - t * e2y, qz = apz - t * e2z;
        return qx * qx + qy * qy + qz * qz;
    }
    float va = d3 * d6 - d5 * d4;
    if (va <= 0.0f && (d4 - d3) >= 0.0f && (d5 - d6) >= 0.0f) {  // edge BC
        float t = (d4 - d3) / ((d4 - d3) + (d5 - d6));
        // q = B + t (C - B);  p - q = bp - t (e2 - e1)
        float qx = bpx - t * (e2x - e1x), qy = bpy - t * (e2y - e1y), qz = bpz - t * (e2z - e1z);
        return qx * qx + qy * qy + qz * qz;
    }
    return s * s;  // face region: distance to the plane
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

// a3 + a4 contact search for a node at predicted position p: candidates are the triangles
// listed in p's cell whose inflated box holds p (ascending id); a candidate is a contact iff
// the point-triangle distance is < thickness, and visit(n, s) is then called with the
// triangle's unit normal n and the signed plane distance s = (p - A).n.  References are
// loaded four at a time (refs has at least four entries of padding) so the ref -> box load
// chains overlap.  Returns the contact count.
template <class Visit>
__device__ __forceinline__ int contacts_visit(const SurfaceView& sv, float px, float py, float pz,
                                              Visit&& visit) {
    const int cell = cell_of(sv, px, py, pz);
    if (cell < 0) return 0;
    const uint32_t b = sv.cell_start[cell], e = sv.cell_start[cell + 1];
    int cnt = 0;
    for (uint32_t r = b; r < e; r += 4) {
        uint32_t t[4];
        float4 lo[4], hi[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) t[q] = sv.refs[r + q];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            lo[q] = sv.box_lo[t[q]];
            hi[q] = sv.box_hi[t[q]];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (r + q < e && in_box(lo[q], hi[q], px, py, pz)) {
                const float4 A = sv.geo[4 * t[q]], e1 = sv.geo[4 * t[q] + 1],
                             e2 = sv.geo[4 * t[q] + 2], n = sv.geo[4 * t[q] + 3];
                const float ax = px - A.x, ay = py - A.y, az = pz - A.z;
                const float s = ax * n.x + ay * n.y + az * n.z;
                const float d2 =
                    point_tri_dist2(ax, ay, az, e1.x, e1.y, e1.z, e2.x, e2.y, e2.z, s);
                if (d2 < sv.thickness2) {
                    visit(n, s);
                    ++cnt;
                }
            }
        }
    }
    return cnt;
}

// Response of Alg. 2 with the averaged direction: with at least one contact, p moves by the
// mean of (th - s_t) n_t over the contacts and q becomes -restitution q.
__device__ __forceinline__ int collide(const SurfaceView& sv, float restitution, float& px,
                                       float& py, float& pz, float& qx, float& qy, float& qz) {
    float sx = 0.0f, sy = 0.0f, sz = 0.0f;
    const float th = sv.thickness;
    const int cnt = contacts_visit(sv, px, py, pz, [&](const float4& n, float s) {
        const float push = th - s;
        sx += push * n.x;
        sy += push * n.y;
        sz += push * n.z;
    });
    if (cnt > 0) {
        const float inv = 1.0f / (float)cnt;
        px += sx * inv;
        py += sy * inv;
        pz += sz * inv;
        qx = -restitution * qx;
        qy = -restitution * qy;
        qz = -restitution * qz;
    }
    return cnt;
}

}  // namespace cloth
