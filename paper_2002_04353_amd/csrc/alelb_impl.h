// Internal declarations shared by the host runtime and the gfx950 kernels of
// the ALE lattice-Boltzmann library.  Not part of the public C-ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace alelb {

constexpr int Q = 9;
constexpr int NPOP = 2 * Q;  // (f_i, g_i) for i = 0..8
constexpr int WALK_CAP = 256;
constexpr double TAU_LOC = 1e-12;  // walk acceptance: min barycentric >= -TAU_LOC
constexpr int BLOCK = 256;
constexpr int NKERNELS = 4;       // streaming, wall fill, k_grad1, k_collide (timed separately)
constexpr int NODES_PER_WAVE = 7;  // k_stream: 7 nodes x 9 directions per wavefront
// every case's node range starts at a multiple of this, so that each k_stream
// workgroup (7 nodes) and each node workgroup (256 nodes) lies inside one case
constexpr int CASE_ALIGN = NODES_PER_WAVE * BLOCK;
// oinfo of a node slot: bits 0-3 slot in the owner element, 4-7 owner-frame
// shift code + 4, bit 8 padding; under the blended pitch law, bit 9 marks a
// node whose departure traces stay inside the rigid zone and bit 10 one whose
// traces stay beyond the blend (there J does not depend on the position)
constexpr uint16_t PAD_NODE = 0x100;
constexpr uint16_t INFO_RIGID = 0x200;
constexpr uint16_t INFO_REST = 0x400;
__host__ __device__ constexpr int info_slot(int info) { return info & 15; }
__host__ __device__ constexpr int info_code(int info) { return (info >> 4) & 15; }

// records the message of the last failure on the calling thread (ale_lb_last_error) and returns code
int report_error(int code, const char *fmt, ...);

// Error word of a handle (device, read back by the host).  Bits 0-2: what
// failed; bit ERR_PARITY + cur: the index of the input buffers of the step
// that failed.  Every step kernel returns at once when the word is set, so
// the first failing step is the only one that raises bits, and the steps
// after it write nothing: its input buffers still hold the last good state.
enum : int { ERR_JAC = 1, ERR_LOCATE = 2, ERR_NONFINITE = 4, ERR_KINDS = 7, ERR_PARITY = 4 };
__host__ __device__ constexpr int err_bits(int kind, int cur) { return kind | (1 << (ERR_PARITY + cur)); }

// time-dependent factors of the motion law at one time level
struct MotionTime {
    double s, c;    // SINE: sin, cos(2 pi t / Tp); PITCH: sin theta, cos theta
    double thd;     // PITCH: dtheta/dt
    double yoff;    // PLUNGE / PITCH: plunge displacement (0, yoff)
    double vy;      // PLUNGE / PITCH: plunge velocity
    double iw;      // PITCH: 1 / (r1 - r0) of the blend (0 without one)
};

struct Motion {
    int kind;
    double p[12];
};

struct Phys {
    double dt, mu, gamma, Pr, Cv, Cp, iCv;  // iCv = 1 / Cv
    double rho_inf, ux_inf, uy_inf, T_inf;
    double chord, refx, refy;
    double Lx, Ly;  // periodic lengths of the case's mesh (0 = not periodic)
};

// The populations are stored as deviations from a per-case reference: the
// case's free-stream equilibrium rounded to a grid coarse enough (multiples of
// 2^-20 for FP32 storage, 2^-44 for FP64) that the reference's moments are
// exact in the storage precision.  In FP32 a stored population then carries
// the rounding of its deviation, not of its full value: the stores of every
// step no longer add an error of a fixed fraction of an ulp of the
// population where the flow lingers.  With exact reference moments the
// moments of a node carry no fixed offset either (an offset in the density
// would be relaxed into the populations at every step).  Entries 0..17 hold
// the reference (f_i, g_i), then its moments, then the far field's missing
// populations as deviations (the free-stream equilibrium minus the
// reference, rounded).
enum {
    REF_RHO = NPOP,  // sum f_i
    REF_JX,          // sum c_ix f_i
    REF_JY,
    REF_PXX,         // sum c_ix c_ix f_i
    REF_PXY,
    REF_PYY,
    REF_SG,          // sum g_i
    REF_FAR = 32,    // 18 entries
    REF_LEN = REF_FAR + NPOP
};

// per-case constants (one entry per case of a batch; a single mesh is one case)
struct CaseStatic {
    Phys ph;
    Motion mo;
    double finf[NPOP];  // free-stream equilibrium (f_i, g_i)
    float ref32[REF_LEN];   // the reference of FP32 storage
    double ref64[REF_LEN];  // the reference of FP64 storage
};

// per-case clock of the step in flight, written by the step before it (or by
// k_clock when the host sets a time)
struct CaseClock {
    double t;          // t^{n+1}: time of the state the step produces
    long long step;    // n + 1: steps completed once the step is done
    MotionTime th;     // factors at t^{n+1/2}
    MotionTime t1;     // factors at t^{n+1}
};

// One element: geometry, neighbours and nodes together, so that a walk step
// and the gather that ends it read one 96-byte record.
struct alignas(16) ElemRec {
    double2 v0;    // vertex 0 in the element frame
    double2 a01;   // (A0, A1): l1 = A0 (x - x0) + A1 (y - y0)
    double2 a23;   // (A2, A3): l2 = A2 (x - x0) + A3 (y - y0)
    int4 nb;       // neighbours across edges 0..2, then pshift codes + 4, 4 bits each
    int n[6];      // nodes v0 v1 v2 m12 m20 m01
    int pad[2];
};

// The part of a triangle's record that the node kernels need (the gradient
// of the shape functions and the node ids), kept apart so that they fetch 64
// of its bytes per owner element instead of 96.
struct alignas(16) ElemGrad {
    double2 a01, a23;  // as in ElemRec
    int n[6];          // as in ElemRec
    int pad[2];
};

// The same coefficients rounded to FP32, for the correction passes of an FP32
// state (40 bytes per owner element): W and X are stored in FP32 there, and
// the coefficients' rounding (a relative 6e-8) is below that of the stored
// values.
struct alignas(8) ElemGradF {
    float2 a01, a23;
    int n[6];
};

// One 9-node quadrilateral (bilinear geometry from the corners): the walk
// reads the corners, neighbours and area, the gather the node ids; 128 bytes.
struct alignas(16) ElemRecQ {
    double2 c[4];  // corners 0..3 in the element frame, counter-clockwise
    int4 nb;       // neighbours across edges 0..3 (edge k: corner k to corner k+1)
    int n[9];      // nodes: corners 0..3, edge nodes 4..7 (node 4+k on edge k), centre 8
    int codes;     // pshift codes + 4 of edges 0..3, 4 bits each
    double a2;     // twice the area
};

enum ElemKind : int { ELEM_P2 = 0, ELEM_Q2 = 1 };

// Device-resident meshes of all cases, concatenated, in the library's internal
// (per-case Hilbert) order.
struct DevMesh {
    int N;                   // node slots including padding
    int E, NW, NWE, ncases;
    int kind;                // ElemKind of every element
    const double2 *X;        // [N] canonical computational coordinates
    const int *own;          // [N] owner element
    const uint16_t *oinfo;   // [N] slot in the owner, owner-frame shift code, padding and zone bits
    const uint8_t *ncase;    // [N] case of each node slot
    const int *wid;          // [N] wall-node index or -1
    const ElemRec *el;       // [E] P2 triangles (kind ELEM_P2)
    const ElemRecQ *elq;     // [E] Q2 quadrilaterals (kind ELEM_Q2)
    const ElemGrad *elg;     // [E] P2: gradient coefficients and node ids of el
    const ElemGradF *elgf;   // [E] P2 with an FP32 state: elg rounded to FP32, else null
    const float2 *Xf;        // [N] P2 with an FP32 state: X rounded to FP32, else null
    const int *bel;          // [NW] element holding point B of each wall node
    const double *blam;      // [3 NW] local coordinates of B: barycentrics, or (xi, eta, 0)
    const int2 *wedge;       // [NWE] (element, local edge)
    const double4 *wxy;      // [NWE] the edge's two vertices (x_a, y_a, x_b, y_b) in the element frame
    const int4 *fblk;        // [force blocks] (case, first wall edge, end wall edge, 0)
};

template <typename R>
struct DevState {
    // [N][9][2] populations (f_i, g_i), ping-pong.  The one-wave schedules
    // store the post-collision populations f*, g*.  The tile schedules store
    // g* and the part of f* the node's own moments fix,
    // f'_i = f~_i + w (f^eq_i - f~_i); the correction phi_i = A_ia X_a is
    // added when the next step stages them: f*_i = f'_i + dt A_ia X_a, X in Xs.
    R *pop[2];
    R *ft;         // [N][9][2] streamed populations
    R *mac[2];     // [N][4] rho ux uy T, ping-pong (previous step / this step)
    R *W;          // [N][2]
    R *Xc;         // [N][2] correction field X_a of the one-wave schedules (kept for tests)
    R *Xs[2];      // [N][2] correction field X_a of the tile schedules, ping-pong like pop
    int *mask;     // [N] missing masks (wall bits 0-8, far-field bits 16-24), optional
    int *err;      // [1] error bits
    int *hint;     // [N][9] element the walk of (node, direction) starts from << 4 | frame code of the
                   // node in that element (periodic shift, (sx+1) + 3 (sy+1)); updated by the walks
    int2 *wlist;   // [N] nodes with wall-crossing directions this step: (node, direction bits)
    int *wcount;   // [1] length of wlist (appended by the streaming kernel, reset by k_collide)
};

template <typename R>
struct StepArgs {
    DevMesh m;
    DevState<R> s;  // wlist / wcount: the list and counter of this launch's node range
    int cur;       // index of the current (input) population / macro buffer
    int flags;     // ALE_LB_F_* of the handle
    int node0, node1;  // node slots of this launch: whole cases, multiples of CASE_ALIGN
    int c0, c1;        // the cases those slots hold
    CaseClock *clock_next;  // the next step's clock of every case, written by this step's k_wall
};

// Tables of the tile kernel, built once on the host.  Nodes are cut into
// tiles of T consecutive (Hilbert-ordered) slots, one workgroup of T threads
// each, one thread per node.  A tile's patch is every element holding one of
// its nodes (rings = 1), optionally with those elements' neighbours
// (rings = 2), and every node of those elements, the tile's own nodes first.
// The workgroup copies the patch into LDS (element records as they are
// stored here, populations through the patch node list) and walks and
// gathers there; a walk that leaves the patch goes on in global memory, and a
// tile whose patch exceeds the LDS budget runs the global path throughout.
//
// Element record, four 16-byte words: v0, (A0, A1), (A2, A3) as in ElemRec,
// then the topology: x = local nodes 0..2, y = local nodes 3..5 (10 bits
// each), z = local neighbours across edges 0..2 (10 bits each: a patch
// element, or TL_OUT / TL_WALL / TL_FAR), w = the edges' shift codes + 4 (4
// bits each).
constexpr unsigned TL_OUT = 1020, TL_WALL = 1021, TL_FAR = 1022;
constexpr int TILE_MAX_LOCAL = 1020;  // patch nodes and patch elements per tile
struct TileArgs {
    const int4 *hdr;    // [tiles] (first patch element, patch elements or -1, first patch node, patch nodes)
    const uint4 *rec;   // [4 per patch element] records as above
    const int *pelem;   // [patch elements] global element id
    const int *pnode;   // [patch nodes] node slot
    const uint4 *start;    // [node slots] start of each direction's walk (10 bits each, local element
                           // index): directions 0-2 in x, 3-5 in y, 6-8 in z; the owner in w
    int pe_max, pn_max;
    int tile;           // nodes per tile
};

// launch schedule: streaming kernel variant and block size of the node kernels
struct Schedule {
    int waves;         // 0: one-wave streaming kernel (global walks and gathers, k_collide);
                       // 2, 4: tile kernel of 64 * waves threads = nodes per tile (LDS patches, split
                       // collision, k_grad2)
    int rings;         // tile kernel: patch radius (1 or 2)
    int node_block;    // k_grad1 / k_collide / k_grad2 workgroup size: 64, 128 or 256
    int groups = 1;    // waves = 0: groups of 7 nodes per workgroup (1, 4, 8), sharing the node metric phase
};
__host__ __device__ constexpr bool tiled(const Schedule &s) { return s.waves != 0; }

constexpr int PATCH_LDS_LIMIT = 80 * 1024;  // dynamic LDS per tile workgroup: two fit a 160 KiB CU
constexpr int TILE_METRIC_BYTES = 56;       // per tile node: J (4), v_g (2), 1 / det J
size_t tile_lds_bytes(int pe_max, int pn_max, int pop_bytes, int T);

template <typename R>
hipError_t launch_step(const StepArgs<R> &a, const CaseStatic *cs, CaseClock *cc, int motion_kind,
                       const Schedule &sch, const TileArgs *ta, hipStream_t st, hipEvent_t *ev);

// the streaming kernel alone (schedule tuning), over a state whose clock was advanced
template <typename R>
hipError_t launch_stream_only(const StepArgs<R> &a, const CaseStatic *cs, const CaseClock *cc, int motion_kind,
                              const Schedule &sch, const TileArgs *ta, hipStream_t st);
template <typename R>
hipError_t launch_node_kernels_only(const StepArgs<R> &a, const CaseStatic *cs, const CaseClock *cc,
                                    int motion_kind, const Schedule &sch, hipStream_t st);

hipError_t launch_clock(const CaseStatic *cs, CaseClock *cc, int ncases, hipStream_t st);

// the two phases of a step over a's node range, for launches that overlap
// one range's streaming with another's node kernels: clock + streaming, then
// wall fill + k_grad1 + k_collide (the one-wave streaming schedule only)
template <typename R>
hipError_t launch_stream_phase(const StepArgs<R> &a, const CaseStatic *cs, CaseClock *cc, int motion_kind,
                               const Schedule &sch, const TileArgs *ta, hipStream_t st);
// the node phase in two parts: the wall fill (the last kernel of a step that
// can raise an error), then the correction passes (and the collision of the
// one-wave schedules)
template <typename R>
hipError_t launch_wall_phase(const StepArgs<R> &a, const CaseStatic *cs, const CaseClock *cc, int motion_kind,
                             const Schedule &sch, hipStream_t st);
template <typename R>
hipError_t launch_grad_phase(const StepArgs<R> &a, const CaseStatic *cs, const CaseClock *cc, int motion_kind,
                             const Schedule &sch, hipStream_t st);
hipError_t launch_freestream(CaseStatic *cs, int ncases, hipStream_t st);

template <typename R>
hipError_t launch_init(const DevMesh &m, DevState<R> s, const CaseStatic *cs, const double *rho,
                       const double *ux, const double *uy, const double *T, int cur, hipStream_t st);

// f'_i + dt A_ia X_a into the populations (tile state -> post-collision state), in place,
// with the arithmetic of the tile kernel's staging; X is then cleared
template <typename R>
hipError_t launch_fold_x(const DevMesh &m, R *pop, R *X, const CaseStatic *cs, hipStream_t st);

hipError_t launch_move_mesh(const DevMesh &m, const CaseStatic *cs, const double *t_case, double *x,
                            double *Jinv, double *det, double *vg, int *err, hipStream_t st);

template <typename R>
hipError_t launch_forces(const DevMesh &m, const R *mac, const CaseStatic *cs, const CaseClock *cc,
                         double *partial, int nblocks, const int2 *case_blocks, double *out, hipStream_t st);

// node-major [n][C] device array of R  <->  component-major [C][n] FP64.
// With m and cs the array holds populations (C = 18), stored as deviations
// from the case's reference: FP64 values are full populations.  With X as
// well (the tile state) they are the post-collision populations
// f'_i + dt A_ia X_a.
template <typename R>
hipError_t launch_convert(const R *src, double *dst, size_t n, int C, hipStream_t st, const DevMesh *m = nullptr,
                          const CaseStatic *cs = nullptr, const R *X = nullptr);
template <typename R>
hipError_t launch_convert_back(const double *src, R *dst, size_t n, int C, hipStream_t st,
                               const DevMesh *m = nullptr, const CaseStatic *cs = nullptr);

}  // namespace alelb
