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

// Device-resident mesh in the library's internal (Morton) order.
struct DevMesh {
    int N, E, NW, NWE;
    double Lx, Ly;
    const double2 *X;        // [N] canonical computational coordinates
    const int *own;          // [N] owner element
    const uint8_t *oinfo;    // [N] bits 0-2: slot in the owner, bits 3-6: owner-frame shift code + 4
    const int *wid;          // [N] wall-node index or -1
    const double2 *eg;       // [3E]: (v0x, v0y), (A0, A1), (A2, A3): (l1, l2) = A (P - v0)
    const int *en;           // [6E] element nodes
    const int4 *et;          // [E] (nbr0, nbr1, nbr2, pshift codes + 4 packed 4 bits each)
    const int *bel;          // [NW] element holding point B of each wall node
    const double *blam;      // [3 NW] barycentrics of B
    const int2 *wedge;       // [NWE] (element, local edge)
    const double4 *wxy;      // [NWE] the edge's two vertices (x_a, y_a, x_b, y_b) in the element frame
};

template <typename R>
struct DevState {
    R *pop[2];     // [18][N] post-collision populations, ping-pong
    R *ft;         // [18][N] streamed populations
    R *mac[2];     // [4][N] rho ux uy T, ping-pong (previous step / this step)
    R *W;          // [2][N]
    R *Xc;         // [2][N] correction field X_a (kept for tests)
    int *mask;     // [N] missing masks (wall bits 0-8, far-field bits 16-24), optional
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
hipError_t launch_init(const DevMesh &m, DevState<R> s, const Phys &ph, const double *rho,
                       const double *ux, const double *uy, const double *T, int cur, hipStream_t st);

hipError_t launch_move_mesh(const DevMesh &m, const Motion &mo, MotionTime tf, double *x,
                            double *Jinv, double *det, double *vg, int *err, hipStream_t st);

template <typename R>
hipError_t launch_forces(const DevMesh &m, const R *mac, const Phys &ph, const Motion &mo,
                         MotionTime tf, double *partial, int nblocks, double *out, hipStream_t st);

template <typename R>
hipError_t launch_convert(const R *src, double *dst, size_t n, hipStream_t st);
template <typename R>
hipError_t launch_convert_back(const double *src, R *dst, size_t n, hipStream_t st);

}  // namespace alelb
