// a3: uniform-grid broad phase over the static surface triangles.
//
// Build (once per surface): per-triangle thickness-inflated boxes and geometry; per-cell
// reference counts by integer atomics; an exclusive prefix sum of the counts built from
// wavefront (64-lane) scans; a scatter of triangle ids into their cells; and a per-cell sort
// so every cell lists its triangles in ascending id (the atomic scatter order is not
// deterministic, the sorted order is).
// Query: a point's cell and an inclusive box test against each triangle listed there; this
// yields exactly the set an all-pairs FP32 box test gives (see cell_coord_f and cell_of).
#include "cloth_device.h"
#include "cloth_internal.h"

namespace cloth {

namespace {

struct Dims {
    float org[3];
    float inv_cell;
    int dim[3];
};

__device__ __forceinline__ void cell_range(const Dims& g, const float4& lo, const float4& hi,
                                           int c0[3], int c1[3]) {
    c0[0] = cell_axis(lo.x, g.org[0], g.inv_cell, g.dim[0]);
    c0[1] = cell_axis(lo.y, g.org[1], g.inv_cell, g.dim[1]);
    c0[2] = cell_axis(lo.z, g.org[2], g.inv_cell, g.dim[2]);
    c1[0] = cell_axis(hi.x, g.org[0], g.inv_cell, g.dim[0]);
    c1[1] = cell_axis(hi.y, g.org[1], g.inv_cell, g.dim[1]);
    c1[2] = cell_axis(hi.z, g.org[2], g.inv_cell, g.dim[2]);
}

Dims make_dims(const float org[3], float inv_cell, const int dim[3]) {
    Dims g;
    for (int a = 0; a < 3; ++a) {
        g.org[a] = org[a];
        g.dim[a] = dim[a];
    }
    g.inv_cell = inv_cell;
    return g;
}

__global__ void k_tri_prep(int T, const float* __restrict__ verts, const int* __restrict__ tris,
                           float th, Dims g, float4* box_lo, float4* box_hi, float4* geo,
                           float4* tri_v, unsigned long long* total_refs) {
#pragma clang fp contract(off)
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    const int ia = tris[3 * t], ib = tris[3 * t + 1], ic = tris[3 * t + 2];
    const float ax = verts[3 * ia], ay = verts[3 * ia + 1], az = verts[3 * ia + 2];
    const float bx = verts[3 * ib], by = verts[3 * ib + 1], bz = verts[3 * ib + 2];
    const float cx = verts[3 * ic], cy = verts[3 * ic + 1], cz = verts[3 * ic + 2];
    float4 lo, hi;
    lo.x = fminf(fminf(ax, bx), cx) - th;
    lo.y = fminf(fminf(ay, by), cy) - th;
    lo.z = fminf(fminf(az, bz), cz) - th;
    lo.w = 0.0f;
    hi.x = fmaxf(fmaxf(ax, bx), cx) + th;
    hi.y = fmaxf(fmaxf(ay, by), cy) + th;
    hi.z = fmaxf(fmaxf(az, bz), cz) + th;
    hi.w = 0.0f;
    box_lo[t] = lo;
    box_hi[t] = hi;
    const float e1x = bx - ax, e1y = by - ay, e1z = bz - az;
    const float e2x = cx - ax, e2y = cy - ay, e2z = cz - az;
    float nx = e1y * e2z - e1z * e2y, ny = e1z * e2x - e1x * e2z, nz = e1x * e2y - e1y * e2x;
    const float len = sqrtf(nx * nx + ny * ny + nz * nz);
    nx /= len;
    ny /= len;
    nz /= len;
    geo[3 * t] = make_float4(ax, ay, az, nx);
    geo[3 * t + 1] = make_float4(e1x, e1y, e1z, ny);
    geo[3 * t + 2] = make_float4(e2x, e2y, e2z, nz);
    tri_v[3 * t] = make_float4(ax, ay, az, __int_as_float(ia));
    tri_v[3 * t + 1] = make_float4(bx, by, bz, __int_as_float(ib));
    tri_v[3 * t + 2] = make_float4(cx, cy, cz, __int_as_float(ic));
    int c0[3], c1[3];
    cell_range(g, lo, hi, c0, c1);
    const unsigned long long n = (unsigned long long)(c1[0] - c0[0] + 1) *
                                 (unsigned long long)(c1[1] - c0[1] + 1) *
                                 (unsigned long long)(c1[2] - c0[2] + 1);
    atomicAdd(total_refs, n);
}

// Workgroup-private counting.  A workgroup's 256 consecutive triangles are usually a compact
// patch of the mesh, so their cell ranges fall in a small box of cells (on the 100,820-
// triangle sphere 97 % of the workgroups' boxes hold at most 8192 cells); when that box holds
// at most kLocalCells cells the workgroup counts its (triangle, cell) pairs with LDS atomics
// and adds one global atomic per touched cell, instead of one per pair (neighbouring
// triangles share cells, and same-address global atomics serialise).  Otherwise it uses
// global atomics per pair.
constexpr int kLocalCells = 8192;

struct Region {
    int lo[3], ext[3];
    int vol;  // 0: the box is empty or too large
};

// Every thread of the workgroup calls this (it synchronises).
__device__ Region block_region(bool valid, const int c0[3], const int c1[3], int* sreg) {
    if (threadIdx.x < 3) {
        sreg[threadIdx.x] = INT_MAX;
        sreg[3 + threadIdx.x] = INT_MIN;
    }
    __syncthreads();
    if (valid)
        for (int a = 0; a < 3; ++a) {
            atomicMin(&sreg[a], c0[a]);
            atomicMax(&sreg[3 + a], c1[a]);
        }
    __syncthreads();
    Region r;
    long long vol = 1;
    for (int a = 0; a < 3; ++a) {
        r.lo[a] = sreg[a];
        r.ext[a] = sreg[3 + a] >= sreg[a] ? sreg[3 + a] - sreg[a] + 1 : 0;
        vol *= r.ext[a];
    }
    r.vol = vol > 0 && vol <= kLocalCells ? (int)vol : 0;
    return r;
}

// Post-increment of a 16-bit LDS counter, through a 32-bit atomic on its aligned word.
__device__ __forceinline__ uint32_t atomic_inc_u16(uint16_t* p) {
    uint32_t* w = reinterpret_cast<uint32_t*>(reinterpret_cast<uintptr_t>(p) & ~(uintptr_t)3);
    const int sh = (reinterpret_cast<uintptr_t>(p) & 2) ? 16 : 0;
    return (atomicAdd(w, 1u << sh) >> sh) & 0xffffu;
}

__device__ __forceinline__ int local_cell(const Region& r, int x, int y, int z) {
    return ((z - r.lo[2]) * r.ext[1] + (y - r.lo[1])) * r.ext[0] + (x - r.lo[0]);
}
__device__ __forceinline__ int global_cell(const Region& r, const Dims& g, int k) {
    const int x = r.lo[0] + k % r.ext[0], y = r.lo[1] + (k / r.ext[0]) % r.ext[1],
              z = r.lo[2] + k / (r.ext[0] * r.ext[1]);
    return (z * g.dim[1] + y) * g.dim[0] + x;
}

__global__ void __launch_bounds__(256)
    k_grid_count(int T, const float4* __restrict__ box_lo, const float4* __restrict__ box_hi,
                 Dims g, uint32_t* counts) {
    __shared__ uint32_t local[kLocalCells];
    __shared__ int sreg[6];
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = t < T;
    int c0[3] = {0, 0, 0}, c1[3] = {-1, -1, -1};
    if (valid) cell_range(g, box_lo[t], box_hi[t], c0, c1);
    const Region r = block_region(valid, c0, c1, sreg);
    if (r.vol == 0) {
        for (int z = c0[2]; z <= c1[2]; ++z)
            for (int y = c0[1]; y <= c1[1]; ++y)
                for (int x = c0[0]; x <= c1[0]; ++x)
                    atomicAdd(&counts[(z * g.dim[1] + y) * g.dim[0] + x], 1u);
        return;
    }
    for (int k = threadIdx.x; k < r.vol; k += blockDim.x) local[k] = 0;
    __syncthreads();
    for (int z = c0[2]; z <= c1[2]; ++z)
        for (int y = c0[1]; y <= c1[1]; ++y)
            for (int x = c0[0]; x <= c1[0]; ++x) atomicAdd(&local[local_cell(r, x, y, z)], 1u);
    __syncthreads();
    for (int k = threadIdx.x; k < r.vol; k += blockDim.x)
        if (local[k]) atomicAdd(&counts[global_cell(r, g, k)], local[k]);
}

// Scatters the triangle ids into their cells' ranges (in an arbitrary order; k_grid_finish
// sorts each cell).  Workgroup-private as k_grid_count: one global atomic per touched cell
// reserves the workgroup's run of slots in that cell.
__global__ void __launch_bounds__(256)
    k_grid_fill(int T, const float4* __restrict__ box_lo, const float4* __restrict__ box_hi,
                Dims g, const uint32_t* __restrict__ cell_start, uint32_t* fill, uint32_t* refs) {
    __shared__ uint32_t local[kLocalCells];  // pair counts, then the run's first slot
    __shared__ __align__(4) uint16_t next[kLocalCells];  // slots taken within the run (<= 256)
    __shared__ int sreg[6];
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = t < T;
    int c0[3] = {0, 0, 0}, c1[3] = {-1, -1, -1};
    if (valid) cell_range(g, box_lo[t], box_hi[t], c0, c1);
    const Region r = block_region(valid, c0, c1, sreg);
    if (r.vol == 0) {
        for (int z = c0[2]; z <= c1[2]; ++z)
            for (int y = c0[1]; y <= c1[1]; ++y)
                for (int x = c0[0]; x <= c1[0]; ++x) {
                    const int c = (z * g.dim[1] + y) * g.dim[0] + x;
                    refs[cell_start[c] + atomicAdd(&fill[c], 1u)] = (uint32_t)t;
                }
        return;
    }
    for (int k = threadIdx.x; k < r.vol; k += blockDim.x) local[k] = next[k] = 0;
    __syncthreads();
    for (int z = c0[2]; z <= c1[2]; ++z)
        for (int y = c0[1]; y <= c1[1]; ++y)
            for (int x = c0[0]; x <= c1[0]; ++x) atomicAdd(&local[local_cell(r, x, y, z)], 1u);
    __syncthreads();
    for (int k = threadIdx.x; k < r.vol; k += blockDim.x)
        if (local[k]) local[k] = atomicAdd(&fill[global_cell(r, g, k)], local[k]);
    __syncthreads();
    for (int z = c0[2]; z <= c1[2]; ++z)
        for (int y = c0[1]; y <= c1[1]; ++y)
            for (int x = c0[0]; x <= c1[0]; ++x) {
                const int k = local_cell(r, x, y, z);
                const int c = (z * g.dim[1] + y) * g.dim[0] + x;
                refs[cell_start[c] + local[k] + atomic_inc_u16(&next[k])] = (uint32_t)t;
            }
}

// One axis of a coded record (see box_code): (Q(lo) + 1) | (0xffff - Q(hi)) << 16 against
// cell coordinate cc, clamped so a corner outside the cell reads as certainly below or
// above every point of it.
__device__ __forceinline__ uint32_t code_axis(float l, float h, float org, float inv_cell,
                                              float cc) {
#pragma clang fp contract(off)
    const float scale = (float)(1 << kCodeBits);
    const float gl = cell_coord_raw(l, org, inv_cell) - cc;
    const float gh = cell_coord_raw(h, org, inv_cell) - cc;
    const float ql = fminf(fmaxf(floorf(gl * scale) + 1.0f, 0.0f), scale);
    const float qh = fminf(fmaxf(floorf(gh * scale), 0.0f), scale);
    return (uint32_t)ql | ((0xffffu - (uint32_t)qh) << 16);
}

// Sorts each cell's reference list ascending and writes the references' records: the
// inflated box inline (ref_lo with the triangle id in .w, ref_hi) and the coded record
// (ref_q).  One wavefront per cell.  A cell lists a triangle at most once, so an entry's
// final position is its rank (the number of smaller entries): up to 128 entries are held
// two per lane and ranked against every entry by broadcasts.  Longer lists (none in
// practice) are insertion-sorted by one lane.
__device__ void finish_cell(int c, int lane, const Dims& g, const uint32_t* __restrict__ cell_start,
                            uint32_t* refs, const float4* __restrict__ box_lo,
                            const float4* __restrict__ box_hi, float4* ref_lo, float4* ref_hi,
                            uint4* ref_q) {
    const uint32_t b = cell_start[c], n = cell_start[c + 1] - b;
    if (n == 0) return;
    const float cc[3] = {(float)(c % g.dim[0]), (float)((c / g.dim[0]) % g.dim[1]),
                         (float)(c / (g.dim[0] * g.dim[1]))};
    auto emit = [&](uint32_t pos, uint32_t t) {
        const float4 lo = box_lo[t], hi = box_hi[t];
        ref_lo[pos] = make_float4(lo.x, lo.y, lo.z, __int_as_float((int)t));
        ref_hi[pos] = hi;
        ref_q[pos] = make_uint4(code_axis(lo.x, hi.x, g.org[0], g.inv_cell, cc[0]),
                                code_axis(lo.y, hi.y, g.org[1], g.inv_cell, cc[1]),
                                code_axis(lo.z, hi.z, g.org[2], g.inv_cell, cc[2]), t);
    };
    if (n <= 128) {
        const uint32_t v0 = lane < (int)n ? refs[b + lane] : 0xffffffffu;
        const uint32_t v1 = lane + 64 < (int)n ? refs[b + 64 + lane] : 0xffffffffu;
        // (entries past n hold 0xffffffff, which is smaller than no entry: the broadcasts
        // stop at the cell's count, which is the same for every lane)
        uint32_t r0 = 0, r1 = 0;
        const int n0 = min((int)n, 64), n1 = (int)n - n0;
        for (int k = 0; k < n0; ++k) {
            const uint32_t w0 = __shfl(v0, k);
            r0 += w0 < v0;
            r1 += w0 < v1;
        }
        for (int k = 0; k < n1; ++k) {
            const uint32_t w1 = __shfl(v1, k);
            r0 += w1 < v0;
            r1 += w1 < v1;
        }
        if (lane < (int)n) {
            refs[b + r0] = v0;
            emit(b + r0, v0);
        }
        if (lane + 64 < (int)n) {
            refs[b + r1] = v1;
            emit(b + r1, v1);
        }
        return;
    }
    if (lane != 0) return;
    for (uint32_t i = b + 1; i < b + n; ++i) {
        const uint32_t v = refs[i];
        uint32_t j = i;
        while (j > b && refs[j - 1] > v) {
            refs[j] = refs[j - 1];
            --j;
        }
        refs[j] = v;
    }
    for (uint32_t i = b; i < b + n; ++i) emit(i, refs[i]);
}

// One wavefront per cell (a bounded grid looping over the cells measured slower).
__global__ void __launch_bounds__(256)
    k_grid_finish(int C, Dims g, const uint32_t* __restrict__ cell_start, uint32_t* refs,
                  const float4* __restrict__ box_lo, const float4* __restrict__ box_hi,
                  float4* ref_lo, float4* ref_hi, uint4* ref_q) {
    const int waves = gridDim.x * (blockDim.x >> 6), lane = threadIdx.x & 63;
    for (int c = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); c < C; c += waves)
        finish_cell(c, lane, g, cell_start, refs, box_lo, box_hi, ref_lo, ref_hi, ref_q);
}

// ------------------------------------------------------------------ prefix sum
// (kScanThreads, kScanItems, kScanTile: cloth_internal.h)

// Inclusive scan across the 64 lanes of a wavefront.
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

// Tile-local exclusive scan of m entries of in (in[n..m) read as 0); sums[tile] = tile total.
__global__ void __launch_bounds__(kScanThreads)
    k_scan_tile(const uint32_t* __restrict__ in, size_t n, size_t m, uint32_t* __restrict__ out,
                uint32_t* __restrict__ sums) {
    __shared__ uint32_t wave_tot[kScanThreads / 64];
    const size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t tot = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        const size_t idx = base + q;
        v[q] = (idx < n) ? in[idx] : 0u;
        tot += v[q];
    }
    const uint32_t incl = wave_inclusive_scan(tot);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 63) wave_tot[wave] = incl;
    __syncthreads();
    if (wave == 0) {
        uint32_t wt = lane < kScanThreads / 64 ? wave_tot[lane] : 0u;
        const uint32_t wi = wave_inclusive_scan(wt);
        if (lane < kScanThreads / 64) wave_tot[lane] = wi - wt;  // exclusive wave offsets
        if (lane == kScanThreads / 64 - 1 && sums) sums[blockIdx.x] = wi;
    }
    __syncthreads();
    uint32_t run = wave_tot[wave] + incl - tot;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        const size_t idx = base + q;
        if (idx < m) out[idx] = run;
        run += v[q];
    }
}

__global__ void __launch_bounds__(kScanThreads)
    k_scan_add(uint32_t* out, size_t m, const uint32_t* __restrict__ offs) {
    const uint32_t add = offs[blockIdx.x];
    const size_t base = (size_t)blockIdx.x * kScanTile;
    for (int q = threadIdx.x; q < kScanTile; q += kScanThreads) {
        const size_t idx = base + q;
        if (idx < m) out[idx] += add;
    }
}

// ------------------------------------------------------------------ point queries
// Broad-phase candidates of arbitrary points through the step kernels' own query
// (contacts_listed, or contacts_visit with hit_slots = 0, stopped before the narrow test):
// the coded box test of each reference of the point's cell, undecided boxes settled with the
// exact box.  One wavefront per workgroup, each lane's hit list in LDS.  WRITE = false
// stores each point's count, WRITE = true its (point, triangle) pairs at its offset.
template <bool WRITE>
__global__ void __launch_bounds__(64)
    k_candidates(int n, int ld, const float* __restrict__ p, SurfaceView sv, int hit_slots,
                 uint32_t* __restrict__ counts, const uint32_t* __restrict__ offsets,
                 int* __restrict__ pairs) {
    extern __shared__ uint32_t hit_lds[];  // wave_query_lds(hit_slots) bytes
    const int i = blockIdx.x * 64 + threadIdx.x;
    if (i >= n) return;
    const float px = p[i], py = p[ld + i], pz = p[2 * ld + i];
    uint32_t o = WRITE ? offsets[i] : 0u;
    auto visit = [&](const float4&, float, uint32_t t) {
        if constexpr (WRITE) {
            pairs[2 * (size_t)o] = i;
            pairs[2 * (size_t)o + 1] = (int)t;
            ++o;
        }
    };
    const int cnt = hit_slots > 0
                        ? contacts_listed<false>(sv, hit_lds + threadIdx.x, hit_slots, px, py, pz, visit)
                        : contacts_visit<false>(sv, px, py, pz, visit);
    if constexpr (!WRITE) counts[i] = (uint32_t)cnt;
}

inline int blocks_for(long long n, int b) { return (int)((n + b - 1) / b); }

}  // namespace

hipError_t launch_tri_prep(int n_tris, const float* verts, const int* tris, float thickness,
                           const float org[3], float inv_cell, const int dim[3], float4* box_lo,
                           float4* box_hi, float4* geo, float4* tri_v,
                           unsigned long long* total_refs, hipStream_t stream) {
    if (n_tris <= 0) return hipSuccess;
    k_tri_prep<<<blocks_for(n_tris, 256), 256, 0, stream>>>(
        n_tris, verts, tris, thickness, make_dims(org, inv_cell, dim), box_lo, box_hi, geo, tri_v,
        total_refs);
    return hipGetLastError();
}

hipError_t launch_grid_count(int n_tris, const float4* box_lo, const float4* box_hi,
                             const float org[3], float inv_cell, const int dim[3],
                             uint32_t* counts, hipStream_t stream) {
    if (n_tris <= 0) return hipSuccess;
    k_grid_count<<<blocks_for(n_tris, 256), 256, 0, stream>>>(
        n_tris, box_lo, box_hi, make_dims(org, inv_cell, dim), counts);
    return hipGetLastError();
}

hipError_t launch_grid_fill(int n_tris, const float4* box_lo, const float4* box_hi,
                            const float org[3], float inv_cell, const int dim[3],
                            const uint32_t* cell_start, uint32_t* fill, uint32_t* refs,
                            hipStream_t stream) {
    if (n_tris <= 0) return hipSuccess;
    k_grid_fill<<<blocks_for(n_tris, 256), 256, 0, stream>>>(
        n_tris, box_lo, box_hi, make_dims(org, inv_cell, dim), cell_start, fill, refs);
    return hipGetLastError();
}

hipError_t launch_grid_finish(int n_cells, const float org[3], float inv_cell, const int dim[3],
                              const uint32_t* cell_start, uint32_t* refs, const float4* box_lo,
                              const float4* box_hi, float4* ref_lo, float4* ref_hi, uint4* ref_q,
                              hipStream_t stream) {
    if (n_cells <= 0) return hipSuccess;
    k_grid_finish<<<blocks_for(n_cells, 4), 256, 0, stream>>>(
        n_cells, make_dims(org, inv_cell, dim), cell_start, refs, box_lo, box_hi, ref_lo, ref_hi,
        ref_q);
    return hipGetLastError();
}

hipError_t scan_exclusive_u32(const uint32_t* in, uint32_t* out, size_t n, uint32_t* tmp,
                              hipStream_t stream) {
    const size_t m = n + 1;
    const size_t nb = (m + kScanTile - 1) / kScanTile;
    uint32_t* sums = tmp;
    k_scan_tile<<<(unsigned)nb, kScanThreads, 0, stream>>>(in, n, m, out, sums);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nb <= 1) return e;
    uint32_t* offs = tmp + nb;
    e = scan_exclusive_u32(sums, offs, nb, tmp + nb + (nb + 1), stream);
    if (e != hipSuccess) return e;
    k_scan_add<<<(unsigned)nb, kScanThreads, 0, stream>>>(out, m, offs);
    return hipGetLastError();
}

hipError_t launch_candidates_count(int n, int ld, const float* p, const SurfaceView& sv,
                                   int hit_slots, uint32_t* counts, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    if (hit_slots < 0 || hit_slots > kMaxHitSlots) return hipErrorInvalidValue;
    k_candidates<false><<<blocks_for(n, 64), 64, wave_query_lds(hit_slots), stream>>>(
        n, ld, p, sv, hit_slots, counts, nullptr, nullptr);
    return hipGetLastError();
}

hipError_t launch_candidates_write(int n, int ld, const float* p, const SurfaceView& sv,
                                   int hit_slots, const uint32_t* offsets, int* pairs,
                                   hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    if (hit_slots < 0 || hit_slots > kMaxHitSlots) return hipErrorInvalidValue;
    k_candidates<true><<<blocks_for(n, 64), 64, wave_query_lds(hit_slots), stream>>>(
        n, ld, p, sv, hit_slots, nullptr, offsets, pairs);
    return hipGetLastError();
}

}  // namespace cloth
