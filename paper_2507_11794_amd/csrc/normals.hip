// Per-vertex cloth normals of the current state (the normal update that precedes shading,
// Sec. 3).  The cloth grid's quads (i, j)-(i+1, j)-(i+1, j+1)-(i, j+1) are split along their
// (i, j)-(i+1, j+1) diagonal into triangles (a, b, c) and (a, c, d); a vertex's normal is the
// normalised sum of (B - A) x (C - A) over its incident triangles (area weighting), so every
// thread that touches a triangle computes the same FP32 cross product.
#include <hip/hip_runtime.h>

#include "cloth_internal.h"

namespace cloth {
namespace {

__device__ __forceinline__ float3 sub(float3 a, float3 b) {
    return make_float3(a.x - b.x, a.y - b.y, a.z - b.z);
}

__device__ __forceinline__ void add_cross(float3 e1, float3 e2, float3& s) {
    s.x += e1.y * e2.z - e1.z * e2.y;
    s.y += e1.z * e2.x - e1.x * e2.z;
    s.z += e1.x * e2.y - e1.y * e2.x;
}

// One thread per internal slot: own position is a coalesced SoA read, the six neighbours
// come from the same or an adjacent 8 x 8 tile; the result goes to caller numbering (AoS).
// Triangles are summed in ascending quad order (row i, then column j), first triangle of a
// quad before the second.
__global__ void k_vertex_normals(int n, int ld, const float* __restrict__ x,
                                 const int* __restrict__ order, const int* __restrict__ slot,
                                 const int* __restrict__ node_group,
                                 const int4* __restrict__ groups, float* __restrict__ out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int4 G = groups[node_group ? node_group[p] : 0];  // node_off, nx, ny, -
    const int id = order[p];
    const int loc = id - G.x, nx = G.y, ny = G.z;
    const int i = loc / nx, j = loc - i * nx;
    const bool up = i > 0, dn = i + 1 < ny, lf = j > 0, rt = j + 1 < nx;
    // neighbours: (i-1, j-1) (i-1, j) (i, j-1) (i, j+1) (i+1, j) (i+1, j+1); missing ones
    // alias the vertex itself and are never used
    const int base = G.x + loc;
    const int s0 = up && lf ? slot[base - nx - 1] : p;
    const int s1 = up ? slot[base - nx] : p;
    const int s2 = lf ? slot[base - 1] : p;
    const int s3 = rt ? slot[base + 1] : p;
    const int s4 = dn ? slot[base + nx] : p;
    const int s5 = dn && rt ? slot[base + nx + 1] : p;
    auto pos = [&](int s) { return make_float3(x[s], x[ld + s], x[2 * ld + s]); };
    const float3 c = pos(p), pul = pos(s0), pu = pos(s1), pl = pos(s2), pr = pos(s3),
                 pd = pos(s4), pdr = pos(s5);
    float3 acc = make_float3(0.0f, 0.0f, 0.0f);
    if (up && lf) {  // quad (i-1, j-1): a = ul, b = l, c = self, d = u
        add_cross(sub(pl, pul), sub(c, pul), acc);
        add_cross(sub(c, pul), sub(pu, pul), acc);
    }
    if (up && rt) add_cross(sub(c, pu), sub(pr, pu), acc);   // quad (i-1, j), first triangle
    if (dn && lf) add_cross(sub(pd, pl), sub(c, pl), acc);   // quad (i, j-1), second triangle
    if (dn && rt) {  // quad (i, j): a = self, b = d, c = dr, d = r
        add_cross(sub(pd, c), sub(pdr, c), acc);
        add_cross(sub(pdr, c), sub(pr, c), acc);
    }
    const float d2 = acc.x * acc.x + acc.y * acc.y + acc.z * acc.z;
    if (d2 > 0.0f) {
        const float len = sqrtf(d2);
        acc.x /= len;
        acc.y /= len;
        acc.z /= len;
    }
    out[3 * (size_t)id + 0] = acc.x;
    out[3 * (size_t)id + 1] = acc.y;
    out[3 * (size_t)id + 2] = acc.z;
}

}  // namespace

hipError_t launch_vertex_normals(int n, int ld, const float* x, const int* order, const int* slot,
                                 const int* node_group, const int4* groups, float* out,
                                 hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_vertex_normals<<<(n + 255) / 256, 256, 0, st>>>(n, ld, x, order, slot, node_group, groups,
                                                      out);
    return hipGetLastError();
}

}  // namespace cloth
