// Spring-centric force accumulation, the form of Alg. 1: one thread per spring computes the
// spring's force and adds +f to end a and -f to end b in an accumulator; a node pass then
// integrates, collides and clears the accumulator for the next substep.  Two accumulators:
//   FIX = false: FP32 atomic adds (the sum order, hence the rounding, varies run to run);
//   FIX = true:  32-bit integer atomics on forces quantised to 2^-24 N (WGSL has only integer
//                atomics, which is why Alg. 2 stores i32 values).  Integer addition commutes,
//                so the result is deterministic; |f| per spring component must stay below
//                8 N (12 incidences per node then stay inside the int32 range), checked per
//                spring (flag bit 2).
// The gather kernels are the default; this path exists to measure the paper's choice.
#include "cloth_device.h"
#include "cloth_internal.h"

namespace cloth {

namespace {

constexpr float kFixScale = 16777216.0f;          // 2^24 LSB per newton
constexpr float kFixInv = 1.0f / 16777216.0f;
constexpr float kFixLimit = 8.0f;                 // newtons per spring and component

template <bool FIX>
__global__ void __launch_bounds__(256)
    k_spring_scatter(const SpringList sl, int ld, const float* __restrict__ xs,
                     const float* __restrict__ vs, float* __restrict__ F, int* flag) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= sl.n) return;
    const int a = sl.a[s], b = sl.b[s];
    float fx = 0.0f, fy = 0.0f, fz = 0.0f;
    spring_force(xs[b] - xs[a], xs[ld + b] - xs[ld + a], xs[2 * ld + b] - xs[2 * ld + a],
                 vs[b] - vs[a], vs[ld + b] - vs[ld + a], vs[2 * ld + b] - vs[2 * ld + a],
                 sl.k[s], sl.c[s], sl.L0[s], fx, fy, fz);
    if (FIX) {
        int* Fi = reinterpret_cast<int*>(F);
        if (!(fabsf(fx) < kFixLimit && fabsf(fy) < kFixLimit && fabsf(fz) < kFixLimit)) {
            atomicOr(flag, 2);
            return;
        }
        const int qx = __float2int_rn(fx * kFixScale), qy = __float2int_rn(fy * kFixScale),
                  qz = __float2int_rn(fz * kFixScale);
        atomicAdd(Fi + a, qx);
        atomicAdd(Fi + ld + a, qy);
        atomicAdd(Fi + 2 * ld + a, qz);
        atomicAdd(Fi + b, -qx);
        atomicAdd(Fi + ld + b, -qy);
        atomicAdd(Fi + 2 * ld + b, -qz);
    } else {
        unsafeAtomicAdd(F + a, fx);
        unsafeAtomicAdd(F + ld + a, fy);
        unsafeAtomicAdd(F + 2 * ld + a, fz);
        unsafeAtomicAdd(F + b, -fx);
        unsafeAtomicAdd(F + ld + b, -fy);
        unsafeAtomicAdd(F + 2 * ld + b, -fz);
    }
}

template <bool FIX, bool COLLIDE, bool GROUPED>
__global__ void __launch_bounds__(256)
    k_node_scatter(const ClothView cv, const StepParams sp, float* __restrict__ F,
                   const float* __restrict__ xs, const float* __restrict__ vs,
                   float* __restrict__ xd, float* __restrict__ vd,
                   const SurfaceView* __restrict__ svs, const int* __restrict__ node_group,
                   const int hit_slots, const int xcd_runs) {
    extern __shared__ uint32_t hit_lds[];  // per wavefront: wave_query_lds(hit_slots) bytes
    const int i = xcd_block(xcd_runs, (cv.n + blockDim.x - 1) / blockDim.x) * blockDim.x +
                  threadIdx.x;
    const bool valid = i < cv.n;
    const int ld = cv.ld;
    float px = 0.0f, py = 0.0f, pz = 0.0f, qx = 0.0f, qy = 0.0f, qz = 0.0f, w = 0.0f;
    if (valid) {
        const float xi = xs[i], yi = xs[ld + i], zi = xs[2 * ld + i];
        const float vxi = vs[i], vyi = vs[ld + i], vzi = vs[2 * ld + i];
        w = cv.w[i];
        float fx, fy, fz;
        if (FIX) {
            const int* Fi = reinterpret_cast<const int*>(F);
            fx = (float)Fi[i] * kFixInv;
            fy = (float)Fi[ld + i] * kFixInv;
            fz = (float)Fi[2 * ld + i] * kFixInv;
        } else {
            fx = F[i];
            fy = F[ld + i];
            fz = F[2 * ld + i];
        }
        F[i] = F[ld + i] = F[2 * ld + i] = 0.0f;  // zero bits: also integer 0
        add_external(sp, i, fx, fy, fz);
        integrate(w, sp.h, sp.g, xi, yi, zi, vxi, vyi, vzi, fx, fy, fz, px, py, pz, qx, qy, qz);
    }
    if (COLLIDE && valid && w != 0.0f) {
        const SurfaceView sv = svs[GROUPED ? node_group[i] : 0];
        if (sv.n_tris > 0) {
            if (hit_slots > 0)
                collide_listed(sv, hit_lds + (threadIdx.x >> 6) * list_stride(hit_slots) + (threadIdx.x & 63),
                               hit_slots, sp.restitution, px, py, pz, qx, qy, qz);
            else
                collide(sv, sp.restitution, px, py, pz, qx, qy, qz);
        }
    }
    if (!valid) return;
    xd[i] = px;
    xd[ld + i] = py;
    xd[2 * ld + i] = pz;
    vd[i] = qx;
    vd[ld + i] = qy;
    vd[2 * ld + i] = qz;
    if (sp.check_nan) {
        const float sum = px + py + pz + qx + qy + qz;
        if (!__builtin_isfinite(sum)) atomicOr(sp.nan_flag, 1);
    }
}

template <bool FIX>
hipError_t launch_nodes(const ClothView& cv, int collide, const StepParams& sp, float* F,
                        const float* xs, const float* vs, float* xd, float* vd, int block,
                        hipStream_t st, const SurfaceView* svs, const int* node_group,
                        int hit_slots, int xcd_runs) {
    if (xcd_runs < 0 || xcd_runs > kMaxXcdRuns) xcd_runs = 0;
    const int grid = xcd_grid((cv.n + block - 1) / block, xcd_runs);
    const size_t lds = collide ? (size_t)(block / 64) * wave_query_lds(hit_slots) : 0;
    if (collide && node_group) {
        k_node_scatter<FIX, true, true><<<grid, block, lds, st>>>(cv, sp, F, xs, vs, xd, vd, svs,
                                                                  node_group, hit_slots, xcd_runs);
    } else if (collide) {
        k_node_scatter<FIX, true, false><<<grid, block, lds, st>>>(cv, sp, F, xs, vs, xd, vd, svs,
                                                                   nullptr, hit_slots, xcd_runs);
    } else {
        k_node_scatter<FIX, false, false><<<grid, block, 0, st>>>(cv, sp, F, xs, vs, xd, vd, svs,
                                                                  nullptr, 0, xcd_runs);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t prepare_scatter_kernels(size_t lds_bytes) {
    if (lds_bytes <= 64 * 1024) return hipSuccess;
    const void* fns[] = {(const void*)k_node_scatter<false, true, false>,
                         (const void*)k_node_scatter<true, true, false>,
                         (const void*)k_node_scatter<false, true, true>,
                         (const void*)k_node_scatter<true, true, true>};
    for (const void* f : fns) {
        const hipError_t e =
            hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_scatter_substep(const ClothView& cv, const SpringList& sl, int fix, int collide,
                                  const StepParams& sp, float* F, const float* xs,
                                  const float* vs, float* xd, float* vd, int block,
                                  hipStream_t st, const SurfaceView* svs, const int* node_group,
                                  int hit_slots, int xcd_runs) {
    if (cv.n <= 0) return hipSuccess;
    if (block <= 0 || block > 256 || (block & 63)) block = 256;
    if (sl.n > 0) {
        const int g = (sl.n + 255) / 256;
        if (fix)
            k_spring_scatter<true><<<g, 256, 0, st>>>(sl, cv.ld, xs, vs, F, sp.nan_flag);
        else
            k_spring_scatter<false><<<g, 256, 0, st>>>(sl, cv.ld, xs, vs, F, sp.nan_flag);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return fix ? launch_nodes<true>(cv, collide, sp, F, xs, vs, xd, vd, block, st, svs,
                                    node_group, hit_slots, xcd_runs)
               : launch_nodes<false>(cv, collide, sp, F, xs, vs, xd, vd, block, st, svs,
                                     node_group, hit_slots, xcd_runs);
}

}  // namespace cloth
