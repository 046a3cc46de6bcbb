// Internal declarations shared by the host runtime and the gfx950 kernels of
// the ALE lattice-Boltzmann library.  Not part of the public C-ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace alelb {

constexpr int Q = 9;
constexpr int NPOP = 2 * Q;  // f_0..f_8, g_0..g_8
constexpr int WALK_CAP = 256;
constexpr double TAU_LOC = 1e-12;  // walk acceptance: min barycentric >= -TAU_LOC
constexpr int BLOCK = 256;
constexpr int NKERNELS = 4;  // k_stream, k_wallbc, k_grad1, k_collide (timed separately)

// error bits raised by the kernels (device word, read back by the host)
enum : int { ERR_JAC = 1, ERR_LOCATE = 2, ERR_NONFINITE = 4 };

// time-dependent factors of the motion law, evaluated once per step on the host
struct MotionTime {
    double s, c;    // SINE: sin, cos(2 pi t / Tp); PITCH: cos theta, sin theta in (c, s)
    double thd;     // PITCH: dtheta/dt
    double yoff;    // PLUNGE / PITCH: plunge displacement (0, yoff)
    double vy;      // PLUNGE / PITCH: plunge velocity
};

struct Motion {
    int kind;
    double p[12];
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

// Device-resident mesh in the library's internal (Morton) order.
struct DevMesh {
    int N, E, NW, NWE;
    int wall_sides;          // element edges tagged as wall (k_wallbc runs when > 0)
    double Lx, Ly;
    const double2 *X;        // [N] canonical computational coordinates
    const int *own;          // [N] owner element
    const uint8_t *oinfo;    // [N] bits 0-2: slot in the owner, bits 3-6: owner-frame shift code + 4
    const int *wid;          // [N] wall-node index or -1
    const ElemRec *el;       // [E]
    const int *bel;          // [NW] element holding point B of each wall node
    const double *blam;      // [3 NW] barycentrics of B
    const int2 *wedge;       // [NWE] (element, local edge)
    const double4 *wxy;      // [NWE] the edge's two vertices (x_a, y_a, x_b, y_b) in the element frame
};

template <typename R>
struct DevState {
    R *pop[2];     // [N][9][2] post-collision populations (f_i, g_i), ping-pong
    R *ft;         // [N][9][2] streamed populations
    R *mac[2];     // [N][4] rho ux uy T, ping-pong (previous step / this step)
    R *W;          // [N][2]
    R *Xc;         // [N][2] correction field X_a (kept for tests)
    int *mask;     // [N] missing masks (wall bits 0-8, far-field bits 16-24), optional
    R *finf;       // [9][2] free-stream equilibrium populations
    int *wl_count; // [1] nodes with a wall-missing direction this step
    int *wl_node;  // [N] their indices
    int *wl_mask;  // [N] their wall-missing direction masks
    int *err;      // [1] error bits
};

struct Phys {
    double dt, mu, gamma, Pr, Cv, Cp;
    double rho_inf, ux_inf, uy_inf, T_inf;
    double chord, refx, refy;
    int flags;
};

template <typename R>
struct StepArgs {
    DevMesh m;
    DevState<R> s;
    Phys ph;
    Motion mo;
    MotionTime th;   // factors at t^{n+1/2}
    MotionTime t1;   // factors at t^{n+1}
    int cur;         // index of the current (input) population / macro buffer
};

MotionTime motion_time(const Motion &mo, double t);

template <typename R>
hipError_t launch_step(const StepArgs<R> &a, hipStream_t st, hipEvent_t *ev);

template <typename R>
hipError_t launch_freestream(const Phys &ph, R *finf, hipStream_t st);

template <typename R>
hipError_t launch_init(const DevMesh &m, DevState<R> s, const Phys &ph, const double *rho,
                       const double *ux, const double *uy, const double *T, int cur, hipStream_t st);

hipError_t launch_move_mesh(const DevMesh &m, const Motion &mo, MotionTime tf, double *x,
                            double *Jinv, double *det, double *vg, int *err, hipStream_t st);

template <typename R>
hipError_t launch_forces(const DevMesh &m, const R *mac, const Phys &ph, const Motion &mo,
                         MotionTime tf, double *partial, int nblocks, double *out, hipStream_t st);

// node-major [n][C] device array of R  <->  component-major [C][n] FP64
template <typename R>
hipError_t launch_convert(const R *src, double *dst, size_t n, int C, hipStream_t st);
template <typename R>
hipError_t launch_convert_back(const double *src, R *dst, size_t n, int C, hipStream_t st);

}  // namespace alelb
