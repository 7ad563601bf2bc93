/*
 * cloth.h -- C ABI of the MI355X (gfx950) mass-spring cloth library.
 *
 * The library advances a mass-spring cloth (Sec. 3 of the paper: nodes joined by springs
 * with rest length, stiffness and damping) through the per-frame path of Sec. 3 and Fig. 2:
 *   1. spring forces of Alg. 1, gathered per node over a CSR incidence list;
 *   2. explicit (semi-implicit Euler) integration with gravity and pinned nodes;
 *   3. a uniform-grid broad phase over the triangles of a static collision surface;
 *   4. point-triangle proximity with a thickness and the averaged response of Alg. 2
 *      (velocity reversed and scaled by the restitution, 0.5 in Alg. 2; position pushed
 *      by the mean of the per-hit directions, Sec. 3 collision paragraph).
 *
 * Conventions (every entry point):
 *   - Return value: CLOTH_OK (0) or a negative CLOTH_E* status.  No call aborts or throws;
 *     cloth_last_error() gives a message for the calling thread's last failure.
 *   - Ownership: the caller owns every array it passes; the library copies inputs at create
 *     time and owns its device memory until the matching destroy.  Host pointers are
 *     marked [host], device pointers [device].
 *   - Layout: host arrays of 3-vectors are AoS, element (i, k) at [i*3 + k], as Alg. 2
 *     writes positions and velocities.  Device state views are SoA, [k*N + i] in the
 *     library's internal node order (see cloth_device_state).
 *   - Streams: every call enqueues on the HIP stream given at create (NULL = the null
 *     stream); calls that return host data synchronise that stream.  A handle is used from
 *     one thread at a time; distinct handles are independent.
 *   - Determinism: for identical inputs the results are bit-identical across runs and
 *     across launch configurations (forces are gathered in a fixed order, no float
 *     atomics; contact sums run in ascending triangle id).
 */
#ifndef CLOTH_H
#define CLOTH_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cloth_sim cloth_sim;     /* opaque, library-owned */
typedef struct cloth_batch cloth_batch; /* opaque, library-owned */

enum cloth_status {
    CLOTH_OK = 0,
    CLOTH_EINVAL = -1,    /* invalid argument or input data */
    CLOTH_ENOMEM = -2,    /* device or host allocation failed, or a size limit was hit */
    CLOTH_EDEVICE = -3,   /* a HIP runtime call or kernel failed */
    CLOTH_EUNSTABLE = -4, /* substep too long for the explicit scheme (see cloth_step) */
    CLOTH_ESTATE = -5,    /* call out of order (e.g. backward without forward) */
    CLOTH_ENAN = -6       /* a non-finite value appeared in the state (CLOTH_F_CHECK_NAN) */
};

/* cloth_params.flags */
#define CLOTH_F_CHECK_NAN 0x1u          /* flag non-finite state values; cloth_read_state
                                           then returns CLOTH_ENAN */
#define CLOTH_F_NO_STABILITY_CHECK 0x2u /* skip the substep-length check of cloth_step */
/* Narrow phase by triangle-triangle intersection (Sec. 3's extended Moller-Trumbore
 * process) instead of point-triangle proximity: surface triangle t is a contact of node i
 * when a cloth edge at i crosses t, an edge of t crosses a cloth triangle at i, or i's path
 * over the substep crosses t (segments oriented from the lower node / vertex id; eps 1e-7).
 * The cloth mesh is the nx-by-ny grid with each quad split along its (i,j)-(i+1,j+1)
 * diagonal.  The response is unchanged (averaged push to the thickness, v <- -r v).  Every
 * substep is then a prediction launch plus a contact launch (the launch configuration's
 * kernel choice does not apply); rollouts are not available on such handles. */
#define CLOTH_F_NARROW_MT 0x4u

typedef struct cloth_params {
    float gravity[3];  /* m/s^2, e.g. {0, -9.81, 0} */
    float thickness;   /* m; contact when point-triangle distance < thickness; 0 disables
                          collision */
    float cell_size;   /* m; broad-phase grid cell edge; <= 0 selects 2 x mean surface edge */
    float restitution; /* on contact v <- -restitution * v (0.5 in Alg. 2) */
    unsigned flags;    /* CLOTH_F_* */
} cloth_params;

/* Launch configuration (cloth_set_launch).  Results are bit-identical for every valid
 * configuration: it changes only how the substeps are scheduled on the GPU. */
enum cloth_kernel {
    CLOTH_KERNEL_TILE = 0,        /* temporally blocked tiles: K substeps per launch in LDS */
    CLOTH_KERNEL_DIRECT = 1,      /* one launch per substep, one thread per node */
    /* spring-centric force accumulation as in Alg. 1 (one thread per spring adding +f / -f
     * to its ends), then a node pass; for measuring the paper's design against the gather */
    CLOTH_KERNEL_SCATTER_F32 = 2, /* FP32 atomic adds: rounding varies from run to run */
    CLOTH_KERNEL_SCATTER_FIX = 3, /* int32 atomics at 2^-24 N (WGSL's integer atomics):
                                     deterministic; |f| < 8 N per spring component, else
                                     cloth_read_state reports CLOTH_ENAN */
    CLOTH_KERNEL_LANES2 = 4,      /* one launch per substep, two lanes per node: each lane
                                     gathers half the node's springs and tests half of its
                                     cell's references (same results as DIRECT, bit for bit) */
    CLOTH_KERNEL_LANES4 = 5,      /* the same with four lanes per node */
    CLOTH_KERNEL_GRID = 6         /* grid cloths whose springs join nodes at most two rows or
                                     columns apart (one spring per offset): one launch per
                                     substep, one wavefront per 8x8 tile of nodes, the tile and
                                     a two-node halo staged in LDS (same results as DIRECT, bit
                                     for bit); block_threads 64, or 128 and more for a second
                                     wavefront per tile that takes every other round of the
                                     box hits' narrow tests (with a surface; same results);
                                     CLOTH_EINVAL for other spring graphs */
};

/* How tiles are assigned to workgroups (tile kernel). */
enum cloth_schedule {
    CLOTH_SCHED_GRID = 0, /* one workgroup per tile, contiguous runs of tiles per XCD */
    CLOTH_SCHED_LPT = 1,  /* `workgroups` persistent workgroups, tiles by decreasing cost to
                             the least-loaded workgroup (longest processing time first) */
    CLOTH_SCHED_RR = 2    /* `workgroups` persistent workgroups, tiles round-robin */
};

typedef struct cloth_launch {
    int kernel;              /* enum cloth_kernel */
    int tile_nodes;          /* tile kernel: nodes per workgroup tile, multiple of 64 (64..4096) */
    int substeps_per_launch; /* tile kernel: substeps advanced per launch, 1..8 */
    int block_threads;       /* threads per workgroup: 64, 128, 192 or 256 (grid kernel: 64
                                one wavefront per tile, 128 and more two) */
    int use_graph;           /* nonzero: replay launches from a captured hipGraph */
    int schedule;            /* tile kernel: enum cloth_schedule */
    int workgroups;          /* persistent schedules: number of workgroups (> 0) */
    int hit_slots;           /* collision query: box hits each node lists in LDS before
                                their geometry is loaded (eight per round; four in the grid
                                kernel when hit_slots <= 16), 0..64; 0 = no
                                list (hits resolved per round of eight references); a node
                                with more hits than slots takes the no-list path (same
                                contacts, same order).  LDS: (hit_slots + 1) * 256 bytes per
                                64 threads. */
    int xcd_runs;            /* one-thread-per-node and grid kernels, 0..4096: how
                                workgroups (node ranges, tiles) map to the 8 XCDs, each with
                                its own L2 (16 by default for grid cloths).  0 keeps
                                the hardware's round-robin order; 1 gives each XCD one
                                contiguous run; k >= 2 deals chunks of k consecutive
                                workgroups to the XCDs in turn */
    int split_refs;          /* one-thread-per-node kernel: nodes whose grid cell lists more
                                than split_refs references are finished by a second launch
                                with four lanes per node (same results); 0 = off */
} cloth_launch;

/*
 * cloth_create -- build a simulation from a cloth grid, its springs and a surface mesh.
 *   nx, ny      grid shape; N = nx*ny nodes, node id i*nx + j for row i, column j (used to
 *               order nodes in memory; any spring graph over the N nodes is accepted).
 *   x0, v0      [host] [N*3] initial positions / velocities (v0 NULL = zero).
 *   mass        [host] [N] node masses, > 0 for unpinned nodes.
 *   pinned      [host] [N] nonzero = pinned node (never moves, zero velocity, no
 *               collision); NULL = none.
 *   n_springs, ends  [host] [S*2] node ids (a, b), a != b; Alg. 1's indexA / indexB.
 *   rest, k, c  [host] [S] rest length > 0, stiffness >= 0, damping >= 0 (Alg. 1).
 *   n_verts, verts   [host] [V*3] surface vertices (may be 0 / NULL).
 *   n_tris, tris     [host] [T*3] vertex ids, wound counter-clockwise seen from outside
 *               (the unit outward normal is normalize((B-A) x (C-A))); no zero-area triangle.
 *   p           [host] parameters, copied.
 *   hip_stream  hipStream_t to run on, or NULL.
 *   out         receives the handle.
 * Errors: CLOTH_EINVAL for N <= 0, S < 0, an index out of range, a == b, rest <= 0,
 *   k < 0, c < 0, mass <= 0 on an unpinned node, any non-finite input, a degenerate
 *   triangle, thickness < 0, restitution outside [0, 1]; CLOTH_ENOMEM; CLOTH_EDEVICE.
 */
int cloth_create(int nx, int ny, const float* x0, const float* v0, const float* mass,
                 const unsigned char* pinned, int n_springs, const int* ends, const float* rest,
                 const float* k, const float* c, int n_verts, const float* verts, int n_tris,
                 const int* tris, const cloth_params* p, void* hip_stream, cloth_sim** out);

/*
 * cloth_step -- advance n_steps frames of length dt, each split into n_substeps substeps
 * of h = dt / n_substeps (forces -> integrate -> broad phase -> narrow phase -> response
 * per substep).  Asynchronous on the handle's stream.
 * Errors: CLOTH_EINVAL (dt <= 0 or non-finite, n_substeps < 1, n_steps < 0);
 *   CLOTH_EUNSTABLE when (w h)^2 + 2 g h >= 4, where w^2 and g bound the largest
 *   eigenvalues of M^-1 K and M^-1 C (Gershgorin row sums of the spring stiffness and
 *   damping matrices at the initial configuration) -- the stability limit of the damped
 *   semi-implicit Euler scheme; skipped with CLOTH_F_NO_STABILITY_CHECK.
 */
int cloth_step(cloth_sim* sim, float dt, int n_substeps, int n_steps);

/*
 * cloth_read_state -- copy the current state to the host, AoS [N*3] in node-id order
 * (Alg. 2's output: updated positions and velocities).  v_out may be NULL.  Synchronises.
 * The state is reordered on the device and copied through a pinned staging buffer that the
 * first call allocates (24 bytes per node of the handle's largest cloth, on the device and
 * in pinned host memory; released by cloth_destroy / cloth_batch_destroy).
 * Returns CLOTH_ENAN if CLOTH_F_CHECK_NAN is set and a non-finite value was produced.
 */
int cloth_read_state(const cloth_sim* sim, float* x_out, float* v_out);

/* cloth_write_state -- overwrite the state from host AoS arrays [N*3] (v may be NULL = 0);
 * with cloth_read_state this gives bit-exact save / resume. */
int cloth_write_state(cloth_sim* sim, const float* x, const float* v);

/*
 * cloth_device_state -- borrowed [device] views of the current state, SoA [3][N] in the
 * library's internal node order, valid until the next cloth_step / cloth_write_state /
 * cloth_destroy.  Either pointer may be NULL.  cloth_node_order gives the order.
 */
int cloth_device_state(cloth_sim* sim, float** x_soa, float** v_soa);

/* cloth_node_order -- [host] [N] out: order[p] = node id stored at internal slot p. */
int cloth_node_order(const cloth_sim* sim, int* order);

/* cloth_info -- sizes: out[0] = N, out[1] = S, out[2] = T, out[3] = grid cells,
 * out[4] = grid references, out[5..7] = grid dims (x, y, z).  [host] out[8]. */
int cloth_info(const cloth_sim* sim, long long* out);

/*
 * cloth_set_launch / cloth_get_launch -- choose how cloth_step schedules substeps.
 * Default when every cloth is a grid whose springs fit the stencil (CLOTH_KERNEL_GRID's
 * condition): the grid kernel, chunks of 16 tiles per XCD, graphs on, 32 hit slots, two
 * wavefronts per tile (block_threads 128) for one cloth with a surface, else one (64).  Otherwise, with a collision surface: the one-thread-per-node
 * kernel, 64 threads per workgroup in the hardware's round-robin order, graphs on, 32 hit
 * slots, no second pass (tile fields: 256 nodes, 1 substep, grid schedule); without one:
 * the tile kernel, 256-node tiles, 1 substep per launch, 256 threads per workgroup, graphs
 * on.
 * cloth_set_launch validates the configuration and rebuilds the tile plan if needed
 * (synchronises the handle's stream).  Errors: CLOTH_EINVAL for an out-of-range field or a
 * tile region that does not fit in LDS (the previous configuration stays in effect).
 */
int cloth_set_launch(cloth_sim* sim, const cloth_launch* cfg);
int cloth_get_launch(const cloth_sim* sim, cloth_launch* cfg);

/* cloth_destroy -- release everything; NULL is accepted. */
int cloth_destroy(cloth_sim* sim);

/*
 * cloth_debug_candidates -- broad-phase candidate pairs of arbitrary query points against
 * the handle's surface grid.  A point P is a candidate of triangle t iff
 * lo_t <= P <= hi_t on every axis, lo_t = fl32(min of t's vertex coordinates - thickness),
 * hi_t = fl32(max + thickness) -- the exact set an O(points x triangles) FP32 brute force
 * gives, found through the uniform grid by the query the step kernels run (the coded box
 * test of the point's cell, undecided boxes settled with the exact box; the handle's
 * hit_slots list length), stopped before the narrow phase.
 *   points     [host] [n_points*3] AoS.
 *   pairs_out  [host] [cap*2] receives (point index, triangle id) sorted by point, then
 *              triangle; at most cap pairs are written.
 *   n_out      [host] receives the total number of pairs (may exceed cap).
 * Errors: CLOTH_EINVAL (n_points < 0, NULL pointers with cap > 0, collision disabled).
 */
int cloth_debug_candidates(cloth_sim* sim, int n_points, const float* points, int* pairs_out,
                           long long cap, long long* n_out);

/*
 * cloth_debug_candidates_noalloc -- cloth_debug_candidates for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments and the same pairs, with the device buffers of the query
 * (the points, their counts and offsets, the scan's partial sums, the pairs) taken from a
 * fixed 8 MiB device array inside the library instead of allocated per call.  No device
 * memory is allocated or freed.  Each GPU the library runs on holds its own copy of that
 * array until the process ends; the call uses the copy of the current device (make the
 * handle's device current), and calls that overlap on one GPU race on it.
 * Limits: n_points <= 65536, and the pairs must fit the rest of the array (786,368
 * pairs at 65,536 points, more for fewer points).
 * Errors: as cloth_debug_candidates; CLOTH_ENOMEM when n_points > 65536 or the pairs do not
 * fit (*n_out then holds the total number of pairs), nothing written to pairs_out.
 */
int cloth_debug_candidates_noalloc(cloth_sim* sim, int n_points, const float* points,
                                   int* pairs_out, long long cap, long long* n_out);

/*
 * cloth_stability_bound -- host-only (no GPU) stability bounds of a spring network at
 * configuration x0: *omega2 and *gamma are the largest Gershgorin row sums of M^-1 K and
 * M^-1 C (K, C assembled from k u u^T and c u u^T per spring, u the unit spring direction);
 * pinned nodes' rows are skipped.  cloth_step rejects h with omega2 h^2 + 2 gamma h >= 4.
 *   x0 [host] [n_nodes*3]; mass [host] [n_nodes]; pinned [host] [n_nodes] or NULL;
 *   ends [host] [S*2]; k, c [host] [S].  Errors: CLOTH_EINVAL as for cloth_create.
 */
int cloth_stability_bound(int n_nodes, const float* x0, const float* mass,
                          const unsigned char* pinned, int n_springs, const int* ends,
                          const float* k, const float* c, double* omega2, double* gamma);

/*
 * cloth_rollout_forward -- differentiable rollout (the gradients of cloth_rollout_backward).
 * Sets the handle's spring stiffness and damping to k, c, starts from the positions given at
 * create and velocities v0, and advances n_steps frames of n_substeps substeps exactly as
 * cloth_step does, recording positions after the frames listed in out_steps and keeping a
 * checkpoint of (x, v) every ckpt_every frames.  The handle's state afterwards is the final
 * rollout state.  Asynchronous on the handle's stream (reads k and c to the host first).
 *   k_dev, c_dev [device] [S] per-spring stiffness and damping, spring-id order.
 *   v0_dev       [device] [N*3] initial velocities, node-id order (NULL = the create-time v0).
 *   out_steps    [host] [n_out] ascending frame counts in 0..n_steps.
 *   x_out_dev    [device] [n_out*N*3] receives the positions at those frames.
 * Memory: (n_steps/ckpt_every + 1) checkpoints, plus ckpt_every*n_substeps + 1 states in
 * the backward pass, N*24 bytes each.
 * Errors: CLOTH_EINVAL (sizes, order, non-finite or negative k / c, a scatter kernel
 * selected: rollouts recompute with the gather kernels), CLOTH_EUNSTABLE.
 */
int cloth_rollout_forward(cloth_sim* sim, const float* k_dev, const float* c_dev,
                          const float* v0_dev, float dt, int n_substeps, int n_steps,
                          int ckpt_every, const int* out_steps, int n_out, float* x_out_dev);

/*
 * cloth_rollout_backward -- gradients of a loss L(x_out) through the last forward rollout,
 * by the exact reverse-mode adjoint of every substep with each node's contact set held at
 * the forward pass's (the derivative of the smooth piece the rollout lies on).
 *   gx_out_dev [device] [n_out*N*3] dL/dx_out.
 *   gk_dev, gc_dev [device] [S] receive dL/dk, dL/dc; gv0_dev [device] [N*3] dL/dv0
 *   (node-id order); any may be NULL.  Gradients accumulate in FP64 per spring.
 * May be called more than once per forward pass.  Asynchronous on the handle's stream.
 * Errors: CLOTH_ESTATE without a preceding successful cloth_rollout_forward.
 */
int cloth_rollout_backward(cloth_sim* sim, const float* gx_out_dev, float* gk_dev,
                           float* gc_dev, float* gv0_dev);

/*
 * cloth_autotune -- measured search over launch configurations for this handle's workload:
 * each candidate (kernel, tile nodes, substeps per launch, threads, schedule) is timed with
 * HIP events over `frames` frames of dt / n_substeps from the current state, which is
 * restored afterwards; the fastest is applied and returned in *best (may be NULL).  Every
 * candidate gives bit-identical results.  If the environment variable CLOTH_AUTOTUNE_CACHE
 * names a file, results are looked up there (keyed by device name and a hash of the
 * workload's sizes) and new results appended.  Synchronises the handle's stream.
 */
int cloth_autotune(cloth_sim* sim, float dt, int n_substeps, int frames, cloth_launch* best);

/* The arguments of cloth_create for one cloth of a batch (borrowed host pointers). */
typedef struct cloth_sim_desc {
    int nx, ny;
    const float* x0;
    const float* v0;
    const float* mass;
    const unsigned char* pinned;
    int n_springs;
    const int* ends;
    const float* rest;
    const float* k;
    const float* c;
    int n_verts;
    const float* verts;
    int n_tris;
    const int* tris;
} cloth_sim_desc;

/*
 * cloth_batch_create -- many independent cloths, each with its own surface, stepped together.
 * descs [host] [n] as for cloth_create (node ids per cloth); p applies to every cloth (with
 * cell_size <= 0 each cloth's grid uses 2 x its own mean surface edge).  All cloths share one
 * node array, one tile plan and one hipGraph; tiles never cross two cloths, so cloth i evolves
 * exactly as a cloth_create handle of its own would (bit for bit).
 * Errors: as cloth_create, for the first invalid cloth (cloth_last_error names it).
 */
int cloth_batch_create(int n, const cloth_sim_desc* descs, const cloth_params* p,
                       void* hip_stream, cloth_batch** out);
/* cloth_batch_step -- cloth_step for every cloth of the batch (stability checked per cloth). */
int cloth_batch_step(cloth_batch* b, float dt, int n_substeps, int n_steps);
/* cloth_batch_read_state -- cloth i's state, AoS [N_i*3] in its own node ids. */
int cloth_batch_read_state(const cloth_batch* b, int i, float* x_out, float* v_out);
/* cloth_batch_set_launch / cloth_batch_get_launch / cloth_batch_autotune -- as for a handle. */
int cloth_batch_set_launch(cloth_batch* b, const cloth_launch* cfg);
int cloth_batch_get_launch(const cloth_batch* b, cloth_launch* cfg);
int cloth_batch_autotune(cloth_batch* b, float dt, int n_substeps, int frames, cloth_launch* best);
/* cloth_batch_info -- out[0] = cloths, out[1] = total nodes, out[2] = total springs,
 * out[3] = total triangles, out[4] = tiles of the current plan, out[5] = workgroups. */
int cloth_batch_info(const cloth_batch* b, long long* out);
/* cloth_batch_destroy -- NULL is accepted. */
int cloth_batch_destroy(cloth_batch* b);

/*
 * cloth_debug_contacts -- the contact set every node would get in a substep of length h
 * from the current state, with the step's own arithmetic: counts[i] triangles, the first
 * min(counts[i], cap) of them (ascending id) at ids[i*cap ...].  counts, ids [host] in node-id
 * order ([N], [N*cap]).  Single-cloth handles.  Synchronises.  With CLOTH_F_NARROW_MT the
 * listed ids are sorted but, past cap, need not be the smallest.
 */
int cloth_debug_contacts(cloth_sim* sim, float h, int* counts, int* ids, int cap);

/*
 * cloth_debug_query_volume -- the surface data the next substep's collision query (a3 with
 * the listed, coded box test of the step kernels) touches from the current state, for
 * counting the collision share of a substep's algorithmic bytes.  out [host] long long[6]:
 *   out[0] distinct non-empty grid cells queried by the unpinned nodes' predictions,
 *   out[1] references listed in those cells (each cell counted once),
 *   out[2] distinct triangles that are a box hit (broad-phase candidate) of some node,
 *   out[3] node queries of a non-empty cell, out[4] references tested over all nodes,
 *   out[5] box hits over all nodes.
 * Single-cloth handles with the proximity narrow phase.  Synchronises.
 * Errors: CLOTH_EINVAL (NULL, h <= 0, batch or MT handle), CLOTH_ESTATE, CLOTH_EDEVICE.
 */
int cloth_debug_query_volume(cloth_sim* sim, float h, long long* out);

/*
 * cloth_update_surface / cloth_batch_update_surface -- move or deform a collision surface:
 * new positions [host] float[n_verts * 3] for the same triangles (n_verts must equal the
 * count given at creation; for a batch, cloth i's surface).  The grid is rebuilt on the
 * device with the cell size fixed at creation; its origin and dims follow the new bounds.
 * Substeps after the call see the new surface (the surface is static between two updates;
 * the response stays v <- -restitution v, not relative to the surface's motion).  Buffers
 * are reused while large enough.  Synchronises the handle's stream (the reference count is
 * read back).  Ends a rollout's validity (CLOTH_ESTATE for a later backward).
 * Errors: CLOTH_EINVAL (NULL, wrong n_verts, non-finite vertex, no collision surface),
 * CLOTH_ENOMEM (grid too fine or too many references; raise cell_size), CLOTH_EDEVICE.
 * A failure after the device arrays started changing leaves the handle refusing to step
 * (CLOTH_ESTATE) until an update of that surface succeeds.
 */
int cloth_update_surface(cloth_sim* sim, const float* verts, int n_verts);
int cloth_batch_update_surface(cloth_batch* b, int i, const float* verts, int n_verts);

/*
 * cloth_set_external_force / cloth_batch_set_external_force -- constant per-node external
 * forces in newtons, f [host] float[N * 3] in node-id order (a batch: all cloths, cloth after
 * cloth), added to the spring forces before integration: v* = v + h (w (F + f) + g) (the
 * pulled-cloth scenes of Sec. 4).  Pinned nodes ignore it.  f = NULL removes the forces.
 * The forces persist until the next call.  Synchronises the handle's stream.
 * Errors: CLOTH_EINVAL (non-finite entry), CLOTH_ENOMEM, CLOTH_EDEVICE.
 */
int cloth_set_external_force(cloth_sim* sim, const float* f);
int cloth_batch_set_external_force(cloth_batch* b, const float* f);

/*
 * cloth_vertex_normals / cloth_batch_vertex_normals -- per-vertex normals of the current
 * cloth state (the normal update before shading, Sec. 3).  Each quad (i,j), (i+1,j),
 * (i+1,j+1), (i,j+1) of the nx-by-ny grid (node (i,j) = i*nx + j) is split along its
 * (i,j)-(i+1,j+1) diagonal into triangles (a,b,c) and (a,c,d); a vertex's normal is the
 * normalised sum of (B-A) x (C-A) over the triangles that contain it (area weighting), or 0
 * if that sum is 0 (e.g. a 1-wide strip).
 * n_out [device] float[3 * N] (N = all nodes of the handle; for a batch, cloth i's nodes
 * follow cloth i-1's), AoS in node-id order; caller-owned, written asynchronously on the
 * handle's stream.  The first call allocates the node-order table (synchronises once).
 * Errors: CLOTH_EINVAL for NULL arguments, CLOTH_EDEVICE for a HIP failure.
 */
int cloth_vertex_normals(cloth_sim* sim, float* n_out);
int cloth_batch_vertex_normals(cloth_batch* b, float* n_out);

/* cloth_status_str -- static text for a status code. */
const char* cloth_status_str(int status);

/* cloth_last_error -- message for the calling thread's last failed call ("" if none). */
const char* cloth_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CLOTH_H */
