/*
 * alelb.h -- C-ABI of the MI355X (gfx950) ALE lattice-Boltzmann hot path.
 *
 * One time step of the arbitrary Lagrangian-Eulerian lattice-Boltzmann solver
 * of Saadat & Karlin ("Arbitrary Lagrangian-Eulerian formulation of lattice
 * Boltzmann model for compressible flows on unstructured moving meshes",
 * arXiv 2002.04353): the two-population compressible D2Q9 model (Sec. IV)
 * propagated semi-Lagrangianly on a fixed computational P2 triangle mesh
 * (Sec. III) along velocities transformed by the moving mesh's Jacobian and
 * grid velocity (Sec. II), with Grad-approximation walls (Sec. IV.A) and the
 * wall force integral (Sec. V.B/V.C coefficients).
 *
 * All functions return an int status: 0 = OK, < 0 = error (ALE_LB_E*); the
 * message of the last failure on the calling thread is ale_lb_last_error().
 * Arrays passed in are caller-owned; create() deep-copies the mesh.  The
 * handle owns every device allocation it makes (hipMalloc) and releases them
 * in ale_lb_destroy().  Every entry point runs on the HIP stream given in
 * ale_lb_params_t.stream (NULL = the null stream) and returns after the
 * stream has drained.
 *
 * Conventions:
 *   D2Q9 velocities, i = 0..8: (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1) (-1,-1) (1,-1).
 *   Populations f_0..f_8 then g_0..g_8; macroscopic fields rho, u_x, u_y, T.
 *   Host-side field and state arrays are structure-of-arrays, FP64, in the
 *   caller's node order (the library reorders nodes internally).
 */
#ifndef ALELB_H
#define ALELB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ale_lb ale_lb_t; /* opaque handle */

enum {
    ALE_LB_OK = 0,
    ALE_LB_EINVAL = -1,       /* bad argument */
    ALE_LB_EMESH = -2,        /* invalid mesh (areas, neighbours, tags, point B outside) */
    ALE_LB_EJAC = -3,         /* mapping Jacobian det <= 0 at a node */
    ALE_LB_ELOCATE = -4,      /* element walk exceeded its step cap */
    ALE_LB_ENONFINITE = -5,   /* non-finite populations detected */
    ALE_LB_EDEVICE = -6,      /* HIP runtime error */
    ALE_LB_ENOMEM = -7,       /* device allocation failed */
    ALE_LB_EUNSUPPORTED = -8  /* unsupported lattice or option */
};

/* motion laws x = G(X, t) (Sec. II; Sec. V.A, eq. Plunge_eq, Sec. V.C)
 *   NONE          x = X
 *   SINE          motion_p = {a, Lx, Ly, Tp}: x = X + d, y = Y + d,
 *                 d = a sin(2 pi X/Lx) sin(2 pi Y/Ly) sin(2 pi t/Tp)
 *   PLUNGE        motion_p = {h, w, phase}: x = X, y = Y - h sin(w t + phase)
 *   PITCH_PLUNGE  motion_p = {A, w, Xc, Yc, phase_p, h, phase_h, r0, r1}:
 *                 x = X + b(r) [R(theta)(X - Xc) + Xc - X + (0, -h sin(w t + phase_h))],
 *                 theta = A sin(w t + phase_p), r = |X - Xc|, b = 1 - s^3 (10 - 15 s + 6 s^2),
 *                 s = clamp((r - r0)/(r1 - r0), 0, 1); r1 <= 0 means b = 1 (rigid). */
enum { ALE_LB_MOTION_NONE = 0, ALE_LB_MOTION_SINE = 1, ALE_LB_MOTION_PLUNGE = 2,
       ALE_LB_MOTION_PITCH_PLUNGE = 3 };

/* precision: FP64 everywhere, or FP32 populations and bulk arithmetic with the
 * departure-point / Jacobian geometry and the force integral kept in FP64 (the
 * correction fields W and X, stored in FP32, take their element gradients
 * and node coordinates from FP32-rounded copies of the geometry).
 * Either way the device stores each population as its deviation from the
 * case's free-stream equilibrium (on a grid whose sums are exact in the
 * storage precision); the state calls take and give full populations. */
enum { ALE_LB_FP64 = 0, ALE_LB_FP32 = 1 };

enum {
    ALE_LB_F_NO_COLLIDE = 1,    /* propagation only (tests): post-collision = streamed */
    ALE_LB_F_CHECK_FINITE = 2,  /* check populations for NaN/Inf every check_every steps */
    ALE_LB_F_KEEP_MASKS = 4,    /* record per-step diagnostics (tests): the missing-direction
                                   masks and the correction field X */
    ALE_LB_F_GRAPH = 8,         /* ale_lb_step replays pairs of steps as one captured HIP graph;
                                   with a NULL stream the handle creates and owns a blocking stream */
    ALE_LB_F_PIPELINE = 16      /* batches of 2+ cases: the cases split at the boundary nearest half
                                   the nodes, and each step runs the halves staggered on the handle's
                                   stream and a second one it owns, the second half's streaming kernel
                                   overlapping the first half's node kernels (takes precedence over
                                   ALE_LB_F_GRAPH).  Every call returns with both streams' work
                                   ordered before later work on the handle's stream. */
};

/* Mesh (Sec. III) on the fixed computational domain, of one element kind:
 * straight-sided 6-node P2 triangles (nv = 6, 3 edges) or 9-node Lagrange
 * quadrilaterals with bilinear geometry (nv = 9, 4 edges; the paper's element).
 *   X          [2*n_nodes] computational coordinates (x0, y0, x1, y1, ...); on a
 *              periodic mesh every node lies in [0, Lx) x [0, Ly).
 *   elem       [nv*n_elems], counter-clockwise.  P2: v0 v1 v2 m12 m20 m01 (node
 *              3+k is the mid-edge node of edge k, opposite vertex k).  Q2:
 *              corners 0..3 at local (xi, eta) = (-1,-1) (1,-1) (1,1) (-1,1),
 *              node 4+k at the middle of edge k (corner k to corner k+1), node 8
 *              at the centre; edge and centre nodes must sit where the bilinear
 *              map of the corners puts them, and every quadrilateral must be
 *              strictly convex.
 *   nbr        [nf*n_elems] element across edge k (nf = 3 or 4); -1 = wall,
 *              -2 = far field.
 *   pshift     [nf*n_elems] periodic shift code crossing edge k, or NULL:
 *              code = (sx+1) + 3 (sy+1) - 4, 0 = none; a point P in the frame of
 *              element e becomes P + (sx Lx, sy Ly) in the frame of nbr[e,k].
 *              The frame of an element puts node 0 at its canonical
 *              coordinates and every other node at its nearest periodic image.
 *   period     (Lx, Ly); zeros for a non-periodic mesh.
 *   wall_edges [2*n_wall_edges] (element, local edge) of every wall edge.
 *   nodes_per_elem  6 (or 0) for P2 triangles, 9 for Q2 quadrilaterals; every
 *              case of a batch has the same kind.  Quadrilateral meshes run
 *              the one-wave streaming schedule (waves = 0). */
typedef struct {
    int32_t n_nodes, n_elems;
    const double *X;
    const int32_t *elem;
    const int32_t *nbr;
    const int8_t *pshift;
    double period[2];
    int32_t n_wall_edges;
    const int32_t *wall_edges;
    int32_t nodes_per_elem;
} ale_lb_mesh_t;

/* lattice and gas (Sec. IV; Sec. V: gamma = 1.4, Pr = 0.71 in the paper).
 * Q must be 9 and shift must be (0, 0); anything else is EUNSUPPORTED. */
typedef struct {
    int32_t Q;
    double gamma, Pr;
    double shift[2];
} ale_lb_lattice_t;

typedef struct {
    double dt, mu;               /* time step; dynamic viscosity (constant) */
    double rho_inf, u_inf[2], T_inf; /* free stream: far-field missing populations, force scaling */
    double chord, ref_point[2];  /* force normalisation length, moment reference point */
    double t0;                   /* time of the initial state */
    int32_t precision;           /* ALE_LB_FP64 or ALE_LB_FP32 */
    int32_t motion;              /* ALE_LB_MOTION_* */
    double motion_p[12];
    int32_t flags;               /* ALE_LB_F_* */
    int32_t check_every;         /* steps between finite/locate checks inside ale_lb_step (0 = end only) */
    void *stream;                /* hipStream_t, NULL = null stream */
    /* Optional device allocator (case 0's is used for a batch; both NULL =
     * hipMalloc / hipFree): dev_alloc(bytes, alloc_ctx) returns device memory
     * on the current device, at least 256-byte aligned, or NULL;
     * dev_free(ptr, alloc_ctx) releases it.  Every device allocation of the
     * handle goes through them: its buffers at create, the tile tables at
     * ale_lb_set_schedule(), the scratch copies of the state and field calls.
     * ale_lb_destroy() returns everything.  EINVAL at create if only one is
     * set or a block is misaligned; ENOMEM if dev_alloc returns NULL (what
     * was taken so far is returned). */
    void *(*dev_alloc)(size_t bytes, void *alloc_ctx);
    void (*dev_free)(void *ptr, void *alloc_ctx);
    void *alloc_ctx;
} ale_lb_params_t;

/* wall forces on the body at the handle's current time: pressure and viscous
 * parts, moments about ref_point (nose-up positive), lift/drag/moment
 * coefficients for a free stream along +x */
typedef struct {
    double F_p[2], F_v[2], M_p, M_v, cl, cd, cm, t;
} ale_lb_forces_t;

/* Validate the mesh (positive areas, strictly convex quadrilaterals with
 * edge and centre nodes at their bilinear positions, symmetric neighbours,
 * consistent wall tags, point B of every wall node inside the mesh), build
 * the owner map
 * (Sec. IV, last paragraph before IV.A), reorder nodes and elements along a
 * Hilbert curve, allocate and upload.  Populations start at zero: call
 * ale_lb_init_fields() or ale_lb_set_state() before stepping. */
int ale_lb_create(const ale_lb_mesh_t *mesh, const ale_lb_lattice_t *lattice,
                  const ale_lb_params_t *params, ale_lb_t **out);

/* A batch of n_cases independent cases (1..255) advanced together by every
 * call: meshes[c] and params[c] describe case c exactly as ale_lb_create()
 * would (Sec. V runs one case each; a batch is an ensemble of such runs, e.g.
 * airfoils at different Mach numbers and motion laws).  The cases may have
 * different meshes, time steps, viscosities, free streams and motion
 * parameters, but must share precision, motion law, flags and stream.  Every
 * case keeps its own clock t_c = t0_c + step * dt_c.  Host-side node arrays of
 * the other entry points concatenate the cases in order (case 0's nodes, then
 * case 1's, ...); ale_lb_get_state() reports case 0's time.  Each case's node
 * range is padded on the device to a multiple of 1792 slots. */
int ale_lb_create_batch(const ale_lb_mesh_t *meshes, const ale_lb_params_t *params, int32_t n_cases,
                        const ale_lb_lattice_t *lattice, ale_lb_t **out);

/* Advance n steps (Sec. II-IV: metrics, departure points, walk, P2 gather,
 * Grad missing populations, moments, two correction passes, collision).
 * Returns after the steps have run and their error word has been read (the
 * call is synchronous; check_every > 0 also reads it every check_every steps
 * inside the call).  If a step fails (EJAC: det J <= 0 at a departure-point
 * metric; ELOCATE: a walk passed its cap of 256 elements; ENONFINITE with
 * ALE_LB_F_CHECK_FINITE: a non-finite population or correction field), the
 * steps after it do nothing and the handle is put back at the last good
 * step: populations, moments, correction field, per-case times and step
 * count are those before the failing step, and the message names both
 * steps.  n = 0 does nothing; EINVAL for n < 0. */
int ale_lb_step(ale_lb_t *h, int32_t n);

/* Physical positions x [2N], inverse Jacobian J^-1 [4N] (row-major), det J [N]
 * and grid velocity [2N] of every node at time t (every case of a batch at
 * the same t) (Sec. II, eq. g_inv).  Any pointer may be NULL.  on_device != 0:
 * the pointers are device pointers of length (padded slots) x components in
 * the library's internal node order; else host pointers in caller order.
 * Returns EJAC if det J <= 0 at any node. */
int ale_lb_move_mesh(ale_lb_t *h, double t, double *x, double *Jinv, double *detJ, double *vg,
                     int32_t on_device);

/* Wall force integral at the current time (FP64 accumulation); for a batch,
 * case 0's forces.  The lift, drag and moment coefficients are those the
 * airfoil cases report (Sec. V.B, plunging airfoil, and Sec. V.C, pitching
 * airfoil): the traction of the pressure p = rho T and of the viscous stress
 * integrated over the wall, divided by (1/2) rho_inf |u_inf|^2 c, the moment
 * about params.ref_point (nose-up positive) by a further c. */
int ale_lb_forces(ale_lb_t *h, ale_lb_forces_t *out);

/* Wall forces of the first n cases of a batch, out[c] for case c (n >= 1;
 * entries beyond the number of cases are left unwritten).  EINVAL for a null
 * handle or out, or n < 1. */
int ale_lb_forces_batch(ale_lb_t *h, ale_lb_forces_t *out, int32_t n);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the wall forces
 * of every case, summed exactly as ale_lb_forces_batch() sums them, written
 * to the caller's device array out_dev[6 * n] as (F_p x, F_p y, F_v x, F_v y,
 * M_p, M_v) per case in case order (the coefficients are these divided by
 * the reference values above).  Enqueued on the handle's stream; the call
 * returns without waiting.  It allocates nothing: the per-workgroup partial
 * sums go to a static device array of the library, 4096 workgroups of 256
 * wall edges (192 KiB per GPU, held until the process ends).  EINVAL for a
 * null argument, n < number of cases, a batch whose wall edges need more than
 * 4096 workgroups, or a current device other than the one the handle was
 * created on.  Every call on a GPU shares that array: calls that overlap on
 * one GPU (two streams, two threads) race. */
int ale_lb_forces_noalloc(ale_lb_t *h, double *out_dev, int32_t n);

/* Current time of the first n cases of a batch (entries beyond the number of
 * cases are left unwritten).  EINVAL for a null handle or t. */
int ale_lb_get_times(ale_lb_t *h, double *t, int32_t n);

/* Set the clock of every case of a batch: t[c] (host, n = number of cases,
 * finite) becomes case c's time, from which the next step's time levels
 * t^{n+1/2}, t^{n+1} of the motion law (Sec. II) are taken.  Restores the
 * per-case times of a checkpoint after ale_lb_set_state(), which gives every
 * case the same time.  EINVAL for a null pointer, n != number of cases or a
 * non-finite time; the handle is then unchanged. */
int ale_lb_set_times(ale_lb_t *h, const double *t, int32_t n);

void ale_lb_destroy(ale_lb_t *h);

/* f = f^eq, g = g^eq of the given fields (Sec. IV eqs. feq, geq_gstar); the
 * fields also become the previous-step macroscopic fields.  Host FP64 arrays
 * of length N in caller order. */
int ale_lb_init_fields(ale_lb_t *h, const double *rho, const double *ux, const double *uy,
                       const double *T);

/* Macroscopic fields of the last completed step.  on_device != 0: device
 * pointers (FP64, internal order, one entry per device node slot); else host
 * pointers in caller order. */
int ale_lb_get_fields(ale_lb_t *h, double *rho, double *ux, double *uy, double *T, int32_t on_device);

/* Checkpoint: post-collision populations pops [18*N], macros [4*N] (host FP64,
 * caller order), time and step counter.  set_state() restores them; in a
 * batch, get_state() reports case 0's time and set_state() gives every case
 * the time t (ale_lb_get_times() / ale_lb_set_times() carry per-case times). */
int ale_lb_get_state(ale_lb_t *h, double *pops, double *macros, double *t, int64_t *step);
int ale_lb_set_state(ale_lb_t *h, const double *pops, const double *macros, double t, int64_t step);

/* Bitwise checkpoint.  The populations are stored as deviations from a
 * per-case reference (the free-stream equilibrium on a coarse grid), so the
 * FP64 values get_state() reports are the stored values plus the reference,
 * rounded: a set_state() of them restarts within FP64 rounding, not bit for
 * bit.  These three carry the state exactly as it is stored.
 *   ale_lb_state_bytes(): size of the blob (negative for a null handle);
 *   ale_lb_save_state(): writes it to host memory buf of `bytes` bytes
 *     (EINVAL if smaller): populations and macros in the storage precision
 *     and internal node order, every case's time and the step counter;
 *   ale_lb_load_state(): restores a blob saved by a handle of the same
 *     precision, meshes and batch (EINVAL otherwise, and the handle is left
 *     unchanged).  The blob does not depend on the launch schedule: a tile
 *     schedule saves its populations with the correction X folded in, as a
 *     switch of schedule family does. */
int64_t ale_lb_state_bytes(ale_lb_t *h);
int ale_lb_save_state(ale_lb_t *h, void *buf, int64_t bytes);
int ale_lb_load_state(ale_lb_t *h, const void *buf, int64_t bytes);

/* Streamed (pre-collision) populations of the last step [18*N] and, when the
 * handle was created with ALE_LB_F_KEEP_MASKS, the missing-direction masks
 * (bit i: direction i crossed a wall / the far field); any pointer may be NULL.
 * Tile schedules (below) record the streamed populations only with
 * ALE_LB_F_KEEP_MASKS: EINVAL for pops otherwise. */
int ale_lb_get_streamed(ale_lb_t *h, double *pops, int32_t *miss_wall, int32_t *miss_far);

/* Correction fields W_a and X_a of the last step [2*N] (Sec. IV eq. Xa); W_a
 * always, X_a always under a tile schedule (it is part of the state there)
 * and with ALE_LB_F_KEEP_MASKS under a one-wave schedule (EINVAL otherwise). */
int ale_lb_get_correction(ale_lb_t *h, double *W, double *Xa);

/* Run n steps with HIP events around every kernel on the handle's stream;
 * ms[k] receives the mean duration of kernel k (0 the streaming kernel:
 * departure points, walk, gather, far-field directions and moments, and on a
 * tile schedule the local part of the collision; 1 Grad wall directions and
 * those nodes' moments; 2 correction pass 1; 3 correction pass 2, with the
 * collision on a one-wave schedule), ms[4] the mean step time.  nk >= 5 and
 * n >= 1, else EINVAL.  The steps advance the state like ale_lb_step(); on a
 * failure ms is left unwritten. */
int ale_lb_time_kernels(ale_lb_t *h, int32_t n, double *ms, int32_t nk);

/* Launch schedule of a step.  Two families:
 *   waves = 0:        one-wave schedules.  The streaming kernel walks and gathers
 *                     in global memory, one 64-lane wavefront per workgroup,
 *                     which takes `groups` groups of 7 consecutive nodes (1, 4
 *                     or 8; 0 = 1): it evaluates the metric at its 7 x groups
 *                     nodes, one lane per node, then runs each group's 7 nodes
 *                     x 9 directions, each walk starting where the last one of
 *                     the same node and direction ended.  The second correction
 *                     pass then forms the post-collision populations in full.
 *   waves = 2, 4:     tile schedules (P2 triangles only).  A tile of 64 x
 *                     waves consecutive (Hilbert-ordered) nodes per workgroup,
 *                     with `groups` threads per node (1, 2 or 3; 0 = 1), each
 *                     taking a third, half or all of the node's nine
 *                     directions.  The tile's patch (elements holding its
 *                     nodes, plus their neighbours when rings = 2, and all
 *                     their nodes) is staged in LDS; each walk starts from a
 *                     table of per-direction start elements in the patch and
 *                     walks and gathers there (on in global memory if it
 *                     leaves the patch), and the node's first thread relaxes
 *                     it with the part of the collision its own moments fix.  The second correction
 *                     pass leaves the correction X_a, which the next step adds
 *                     as it stages the populations.  Tiles whose patch exceeds
 *                     the LDS budget walk and gather in global memory.
 *   node_block:       workgroup size of the per-node kernels (64, 128, 256).
 *   lds_limit:        cap in bytes on the LDS a tile's patch may take, 0 = what
 *                     the device's per-workgroup limit (at most 80 KiB, less
 *                     56 bytes per tile node for the node metrics) leaves;
 *                     a small cap sends tiles to the global path (tests).
 * Within a family every schedule computes the same values in the same order
 * (bit-identical results).  The families agree to round-off: their walks
 * start from different elements, and a departure point on an edge shared by
 * two elements is interpolated in either.  A change of family converts the
 * current state exactly.  Builds the tile tables on the host and uploads them
 * (the handle owns them).  EINVAL for values outside the lists above;
 * EUNSUPPORTED if a tile's output rows do not fit the device's LDS, or for
 * waves other than 0 on quadrilaterals. */
int ale_lb_set_schedule(ale_lb_t *h, int32_t waves, int32_t rings, int32_t node_block, int32_t lds_limit,
                        int32_t groups);

/* Pick the schedule by timing: every variant (waves 0 with groups 1, 4, 8;
 * waves 2, 4 with rings 1 and 2), timed as streaming kernel + correction
 * passes, then node_block 64, 128, 256, each over reps launches on the
 * handle's current state; the state's inputs and clock are left unchanged,
 * the last step's outputs (streamed populations, ...) are overwritten.  The choice is cached in the
 * process per (precision, motion law, element kind, number of cases, log2
 * total nodes, log2 nodes per case); quadrilateral meshes time the one-wave
 * variants only; a later call in the same bucket applies the cached choice
 * without timing.  reps = 0 drops the cached choice of this bucket.
 * choice[6] (may be NULL) receives waves, rings, node_block, 1 if taken from
 * the cache, the number of tiles on the global path, and groups; *ms (may be
 * NULL) the timed streaming + node-kernel time per step. */
int ale_lb_autotune(ale_lb_t *h, int32_t reps, int32_t *choice, double *ms);

/* sizes: out[0] nodes, [1] elements, [2] wall edges, [3] wall nodes,
 * [4] device bytes held, [5] bytes per population scalar, [6] cases,
 * [7] device node slots (nodes plus per-case padding), [8] tiles on the global
 * path under the current schedule; under a tile schedule [9] the largest
 * patch's nodes and [10] elements the LDS layout holds, [11] the dynamic LDS
 * bytes of a tile workgroup (zeros under a one-wave schedule) */
int ale_lb_info(ale_lb_t *h, int64_t *out, int32_t n);

/* internal node order: perm[k] = caller index of internal node k, for the
 * n_nodes caller nodes (padding slots skipped).  EINVAL for a null argument. */
int ale_lb_node_order(ale_lb_t *h, int32_t *perm);

const char *ale_lb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ALELB_H */
