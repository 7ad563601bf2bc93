// Device helpers shared by the HIP kernels: grid cell mapping, inflated-box test, spring
// force of one incidence, and point-triangle closest-point distance.
#pragma once

#include <hip/hip_runtime.h>

#include "cloth_internal.h"

namespace cloth {

// Grid coordinate of one axis.  Monotone non-decreasing in p (each FP32 operation rounds
// to nearest, floor and the clamp are monotone), so a triangle registered in the cells
// spanned by cell(lo)..cell(hi) of its inflated box is found from any point inside the
// box.  NaN maps to 0.  No contraction: the result must match the build bit for bit.
__device__ __forceinline__ int cell_axis(float p, float org, float inv_cell, int dim) {
#pragma clang fp contract(off)
    float f = floorf((p - org) * inv_cell);
    f = fminf(fmaxf(f, 0.0f), (float)(dim - 1));
    return (int)f;
}

__device__ __forceinline__ int cell_of(const SurfaceView& sv, float px, float py, float pz) {
    int cx = cell_axis(px, sv.org[0], sv.inv_cell, sv.dim[0]);
    int cy = cell_axis(py, sv.org[1], sv.inv_cell, sv.dim[1]);
    int cz = cell_axis(pz, sv.org[2], sv.inv_cell, sv.dim[2]);
    return (cz * sv.dim[1] + cy) * sv.dim[0] + cx;
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

}  // namespace cloth
