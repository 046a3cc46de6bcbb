// gfx950 kernels of the ALE lattice-Boltzmann time step (Saadat & Karlin,
// arXiv 2002.04353).  One step is four launches over the nodes of every case
// (a batch of independent meshes, or one mesh), all gathers on an
// unstructured mesh of 6-node P2 triangles or 9-node Q2 quadrilaterals (the
// element kind is a template argument).  Each case's clock (its time and the
// motion-law factors at t^{n+1/2}, t^{n+1}) sits in one of two buffers:
// k_clock primes it, and each step's k_wall writes the next step's.
//
//   k_stream   metrics at t^{n+1/2} and the transformed velocities
//              c^_i = J^-1 (c_i - v_g) (Sec. II, eq. Trasformed_Discrete_Vel),
//              departure points traced by the midpoint rule, element walk
//              (Sec. III, eq. NonLinear_Eq), finite-element gather-interpolation
//              (eq. Propagation), free-stream missing populations and the
//              moments (eq. Temp); nodes with wall-crossing directions are listed
//   k_wall     the listed nodes: Grad missing populations (Sec. IV.A,
//              tab. Neq_Moments) and their moments; the next step's clock
//   k_grad1    W_a = (mu / rho T) d_a Q'_aaa through the owner element
//              (eqs. Xa, DeviationTerms, Ph_Derivative, FE_Derivative).
//   k_collide  X_a = -d_a W_a, then the two-population collision with
//              phi_i = A_ia X_a (eqs. feqn, geqn, feq, geq_gstar, Wi, Ai,
//              tab. Eq_Moments).
//
// R is the type of the populations and of the bulk arithmetic (float or
// double); coordinates, Jacobians, element local coordinates and the force
// integral are always double.  Nodes are Hilbert-ordered; populations are
// node-major [N][9][2] (f_i and g_i adjacent), moments [N][4], correction
// fields [N][2].  A launch covers a range of whole cases (the whole batch,
// or one half of it when the halves run on two streams).
#include <hip/hip_runtime.h>

#include "alelb_impl.h"

namespace alelb {

namespace {

constexpr double PI = 3.14159265358979323846;

// D2Q9 velocity components, packed two bits per direction (value + 1)
constexpr unsigned pack_c(const int (&c)[9])
{
    unsigned r = 0;
    for (int i = 0; i < 9; ++i) r |= unsigned(c[i] + 1) << (2 * i);
    return r;
}
constexpr int CX_[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int CY_[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr unsigned CXP = pack_c(CX_);
constexpr unsigned CYP = pack_c(CY_);

__device__ __forceinline__ int cx_of(int i) { return int((CXP >> (2 * i)) & 3u) - 1; }
__device__ __forceinline__ int cy_of(int i) { return int((CYP >> (2 * i)) & 3u) - 1; }

// 1 / x from the hardware reciprocal refined by two Newton steps: within
// about an ulp of the rounded quotient, for finite non-zero x, at under half
// the instructions of a full IEEE divide (FP64 geometry only)
__device__ __forceinline__ double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// ---- motion law (Sec. II): Jacobian J = dx/dX and grid velocity at (X, Y) ----
// MK is the motion law (ALE_LB_MOTION_*), fixed per kernel instantiation
template <int MK>
__device__ __forceinline__ void metric_k(const Motion &mo, const MotionTime &tf, double X, double Y,
                                         double J[4], double v[2])
{
    J[0] = 1.0; J[1] = 0.0; J[2] = 0.0; J[3] = 1.0;
    v[0] = 0.0; v[1] = 0.0;
    if constexpr (MK == 1) {
        const double a = mo.p[0], Lx = mo.p[1], Ly = mo.p[2], Tp = mo.p[3];
        double sx, cx, sy, cy;
        sincos(2.0 * PI * X / Lx, &sx, &cx);
        sincos(2.0 * PI * Y / Ly, &sy, &cy);
        const double dX = a * (2.0 * PI / Lx) * cx * sy * tf.s;
        const double dY = a * (2.0 * PI / Ly) * sx * cy * tf.s;
        const double dT = a * sx * sy * (2.0 * PI / Tp) * tf.c;
        J[0] = 1.0 + dX; J[1] = dY;
        J[2] = dX;       J[3] = 1.0 + dY;
        v[0] = dT; v[1] = dT;
    } else if constexpr (MK == 2) {
        v[1] = tf.vy;
    } else if constexpr (MK == 3) {
        const double Xc = mo.p[2], Yc = mo.p[3], r0 = mo.p[7], r1 = mo.p[8];
        const double c = tf.c, s = tf.s;
        const double rx = X - Xc, ry = Y - Yc;
        const double Dx = c * rx - s * ry + Xc - X;
        const double Dy = s * rx + c * ry + Yc - Y + tf.yoff;
        const double Vx = tf.thd * (-s * rx - c * ry);
        const double Vy = tf.thd * (c * rx - s * ry) + tf.vy;
        double b = 1.0, bX = 0.0, bY = 0.0;
        if (r1 > 0.0) {
            // The blend is exactly 1 inside r0 and 0 beyond r1.  Squared radii
            // with a 1e-12 relative margin decide those zones without the root
            // and divides; points near either radius take the full formula,
            // so every point gets the value the full formula gives.
            const double r2 = rx * rx + ry * ry;
            if (r2 > r1 * r1 * (1.0 + 1e-12)) {
                b = 0.0;
            } else if (!(r2 < r0 * r0 * (1.0 - 1e-12))) {
                // s = (r - r0) / (r1 - r0), grad b = b'(s) (x - x_c) / (r (r1 - r0)):
                // 1 / (r1 - r0) comes with the time factors, one divide is left
                const double r = sqrt(r2);
                const double sb = (r - r0) * tf.iw;
                if (sb >= 1.0) {
                    b = 0.0;
                } else if (sb > 0.0) {
                    b = 1.0 - sb * sb * sb * (10.0 - 15.0 * sb + 6.0 * sb * sb);
                    const double db = -30.0 * sb * sb * (1.0 - sb) * (1.0 - sb);
                    const double q = db * tf.iw * rcp_nr(r);
                    bX = q * rx;
                    bY = q * ry;
                }
            }
        }
        J[0] = 1.0 + b * (c - 1.0) + Dx * bX;
        J[1] = b * (-s) + Dx * bY;
        J[2] = b * s + Dy * bX;
        J[3] = 1.0 + b * (c - 1.0) + Dy * bY;
        v[0] = b * Vx; v[1] = b * Vy;
    }
}

__device__ __forceinline__ void metric(const Motion &mo, const MotionTime &tf, double X, double Y, double J[4],
                                       double v[2])
{
    switch (mo.kind) {
    case 1: metric_k<1>(mo, tf, X, Y, J, v); break;
    case 2: metric_k<2>(mo, tf, X, Y, J, v); break;
    case 3: metric_k<3>(mo, tf, X, Y, J, v); break;
    default: metric_k<0>(mo, tf, X, Y, J, v); break;
    }
}

__device__ __forceinline__ void position(const Motion &mo, const MotionTime &tf, double X, double Y,
                                         double &x, double &y)
{
    x = X; y = Y;
    if (mo.kind == 1) {
        const double a = mo.p[0], Lx = mo.p[1], Ly = mo.p[2];
        const double d = a * sin(2.0 * PI * X / Lx) * sin(2.0 * PI * Y / Ly) * tf.s;
        x = X + d; y = Y + d;
    } else if (mo.kind == 2) {
        y = Y + tf.yoff;
    } else if (mo.kind == 3) {
        const double Xc = mo.p[2], Yc = mo.p[3], r0 = mo.p[7], r1 = mo.p[8];
        const double rx = X - Xc, ry = Y - Yc;
        const double Dx = tf.c * rx - tf.s * ry + Xc - X;
        const double Dy = tf.s * rx + tf.c * ry + Yc - Y + tf.yoff;
        double b = 1.0;
        if (r1 > 0.0) {
            const double sb = (sqrt(rx * rx + ry * ry) - r0) / (r1 - r0);
            b = sb >= 1.0 ? 0.0 : (sb > 0.0 ? 1.0 - sb * sb * sb * (10.0 - 15.0 * sb + 6.0 * sb * sb) : 1.0);
        }
        x = X + b * Dx; y = Y + b * Dy;
    }
}

// physical gradient g_x = g^-1 g_X with g^-1 = J^-T (Sec. II eq. g_inv; eq. Ph_Derivative)
__device__ __forceinline__ void to_physical(const double J[4], double gX, double gY, double &gx, double &gy)
{
    const double id = rcp_nr(J[0] * J[3] - J[1] * J[2]);
    gx = (J[3] * gX - J[2] * gY) * id;
    gy = (-J[1] * gX + J[0] * gY) * id;
}

// ---- element walk over neighbours; P is updated across periodic edges ----
// One step of the visibility walk in element e with geometry (v0, a01, a23):
// returns true when P lies in e (barycentrics in l), else the edge to cross in k.
__device__ __forceinline__ void barycentric(double2 v0, double2 a01, double2 a23, double Px, double Py, double l[3])
{
    const double dx = Px - v0.x, dy = Py - v0.y;
    l[1] = a01.x * dx + a01.y * dy;
    l[2] = a23.x * dx + a23.y * dy;
    l[0] = 1.0 - l[1] - l[2];
}

__device__ __forceinline__ bool walk_test(double2 v0, double2 a01, double2 a23, double Px, double Py, double l[3],
                                          int &k)
{
    barycentric(v0, a01, a23, Px, Py, l);
    k = 0;
    double mn = l[0];
    if (l[1] < mn) { k = 1; mn = l[1]; }
    if (l[2] < mn) { k = 2; mn = l[2]; }
    return mn >= -TAU_LOC;
}

// cross edge k of an element with neighbour record t; returns the next element or the boundary code
__device__ __forceinline__ int walk_cross(double Lx, double Ly, int4 t, int k, double &Px, double &Py)
{
    const int n = k == 0 ? t.x : (k == 1 ? t.y : t.z);
    if (n < 0) return n;
    const int code = int((unsigned(t.w) >> (4 * k)) & 15u) - 4;
    if (code != 0) {
        const int c = code + 4;
        Px += double(c % 3 - 1) * Lx;
        Py += double(c / 3 - 1) * Ly;
    }
    return n;
}

// walk that reads whole element records: returns the element holding P (>= 0)
// with its barycentrics and node ids, or -1 wall, -2 far field, -4 cap; `last`
// is the last element visited inside the domain
__device__ __forceinline__ int walk_rec(const ElemRec *__restrict__ el, double Lx, double Ly, int e, double &Px,
                                        double &Py, double l[3], int nd[6], int &last)
{
    for (int it = 0; it < WALK_CAP; ++it) {
        const ElemRec &r = el[e];
        const double2 v0 = r.v0, a01 = r.a01, a23 = r.a23;
        const int4 nb = r.nb;
        const int4 n03 = *reinterpret_cast<const int4 *>(&r.n[0]);
        const int2 n45 = *reinterpret_cast<const int2 *>(&r.n[4]);
        int k;
        last = e;
        if (walk_test(v0, a01, a23, Px, Py, l, k)) {
            nd[0] = n03.x; nd[1] = n03.y; nd[2] = n03.z; nd[3] = n03.w; nd[4] = n45.x; nd[5] = n45.y;
            return e;
        }
        e = walk_cross(Lx, Ly, nb, k, Px, Py);
        if (e < 0) return e;
    }
    return -4;
}

// Frame code of a node in the frame of the element its departure point was
// found in (periodic meshes: the walk shifts the point as it crosses periodic
// edges).  With `recompute`, the point is then formed again in that frame from
// the node's canonical coordinates, with its barycentrics, so that the result
// does not depend on the path the walk took.
__device__ __forceinline__ int frame_code(double Lx, double Ly, double2 Xa, double dt, double chx, double chy,
                                          double Px, double Py)
{
    const int sx = Lx > 0.0 ? int(rint((Px + dt * chx - Xa.x) / Lx)) : 0;
    const int sy = Ly > 0.0 ? int(rint((Py + dt * chy - Xa.y) / Ly)) : 0;
    return (sx + 1) + 3 * (sy + 1);
}
__device__ __forceinline__ void reframe(const ElemRec &r, double Lx, double Ly, double2 Xa, double dt, double chx,
                                        double chy, int code, double l[3])
{
    const double Px = (Xa.x + double(code % 3 - 1) * Lx) - dt * chx;
    const double Py = (Xa.y + double(code / 3 - 1) * Ly) - dt * chy;
    barycentric(r.v0, r.a01, r.a23, Px, Py, l);
}

// P2 shape functions: N_k = l_k (2 l_k - 1), N_{3+k} = 4 l_{k+1} l_{k+2}
__device__ __forceinline__ void p2_shape(const double l[3], double N[6])
{
    N[0] = l[0] * (2.0 * l[0] - 1.0);
    N[1] = l[1] * (2.0 * l[1] - 1.0);
    N[2] = l[2] * (2.0 * l[2] - 1.0);
    N[3] = 4.0 * l[1] * l[2];
    N[4] = 4.0 * l[2] * l[0];
    N[5] = 4.0 * l[0] * l[1];
}

// gradients (computational) of the six P2 shape functions at local node `slot`
__device__ __forceinline__ void p2_grad_at_node(int slot, double2 a01, double2 a23, double gN[6][2])
{
    const double gl[3][2] = {{-a01.x - a23.x, -a01.y - a23.y}, {a01.x, a01.y}, {a23.x, a23.y}};
    // barycentrics of the node: 1 at its own vertex, 1/2 at both ends of its edge
    double l[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) l[k] = slot == k ? 1.0 : ((slot >= 3 && slot != 3 + k) ? 0.5 : 0.0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            gN[k][d] = (4.0 * l[k] - 1.0) * gl[k][d];
            gN[3 + k][d] = 4.0 * (l[k1] * gl[k2][d] + l[k2] * gl[k1][d]);
        }
    }
}

// ---- 9-node quadrilateral (Sec. III): tensor Lagrange interpolation on
// [-1,1]^2 over the bilinear map of the corners ----
// local coordinates of the nodes, (xi_s + 1) and (eta_s + 1) in 2 bits each:
// corners (-1,-1) (1,-1) (1,1) (-1,1), edge nodes (0,-1) (1,0) (0,1) (-1,0), centre (0,0)
constexpr uint32_t QXIP = 0u | 2u << 2 | 2u << 4 | 0u << 6 | 1u << 8 | 2u << 10 | 1u << 12 | 0u << 14 | 1u << 16;
constexpr uint32_t QETP = 0u | 0u << 2 | 2u << 4 | 2u << 6 | 0u << 8 | 1u << 10 | 2u << 12 | 1u << 14 | 1u << 16;
__host__ __device__ constexpr int q_xi(int s) { return int((QXIP >> (2 * s)) & 3u) - 1; }
__host__ __device__ constexpr int q_eta(int s) { return int((QETP >> (2 * s)) & 3u) - 1; }

// 1-D quadratic Lagrange basis on the nodes -1, 0, 1 and its derivative
__device__ __forceinline__ void lagrange3(double t, double L[3], double dL[3])
{
    L[0] = 0.5 * t * (t - 1.0);
    L[1] = (1.0 - t) * (1.0 + t);
    L[2] = 0.5 * t * (t + 1.0);
    dL[0] = t - 0.5;
    dL[1] = -2.0 * t;
    dL[2] = t + 0.5;
}

// N_s(xi, eta) = L_{xi_s}(xi) L_{eta_s}(eta)
__device__ __forceinline__ void q2_shape(const double l[3], double N[9])
{
    double Lx[3], Ly[3], d[3];
    lagrange3(l[0], Lx, d);
    lagrange3(l[1], Ly, d);
#pragma unroll
    for (int s = 0; s < 9; ++s) N[s] = Lx[q_xi(s) + 1] * Ly[q_eta(s) + 1];
}

// bilinear map x = b0 + b1 xi + b2 eta + b3 xi eta of corners c0..c3
struct Bilinear {
    double2 b0, b1, b2, b3;
};
__device__ __forceinline__ Bilinear bilinear(const ElemRecQ &r)
{
    const double2 c0 = r.c[0], c1 = r.c[1], c2 = r.c[2], c3 = r.c[3];
    Bilinear B;
    B.b0 = make_double2(0.25 * (c0.x + c1.x + c2.x + c3.x), 0.25 * (c0.y + c1.y + c2.y + c3.y));
    B.b1 = make_double2(0.25 * (-c0.x + c1.x + c2.x - c3.x), 0.25 * (-c0.y + c1.y + c2.y - c3.y));
    B.b2 = make_double2(0.25 * (-c0.x - c1.x + c2.x + c3.x), 0.25 * (-c0.y - c1.y + c2.y + c3.y));
    B.b3 = make_double2(0.25 * (c0.x - c1.x + c2.x - c3.x), 0.25 * (c0.y - c1.y + c2.y - c3.y));
    return B;
}

// eq. NonLinear_Eq: (xi, eta) with x(xi, eta) = P, by Newton's method from the
// centre (at most 8 iterations, stopping once the update is below 1e-14)
__device__ __forceinline__ void q2_local(const ElemRecQ &r, double Px, double Py, double l[3])
{
    const Bilinear B = bilinear(r);
    double xi = 0.0, eta = 0.0;
    for (int it = 0; it < 8; ++it) {
        const double rx = B.b0.x + B.b1.x * xi + B.b2.x * eta + B.b3.x * xi * eta - Px;
        const double ry = B.b0.y + B.b1.y * xi + B.b2.y * eta + B.b3.y * xi * eta - Py;
        const double j00 = B.b1.x + B.b3.x * eta, j01 = B.b2.x + B.b3.x * xi;
        const double j10 = B.b1.y + B.b3.y * eta, j11 = B.b2.y + B.b3.y * xi;
        const double id = rcp_nr(j00 * j11 - j01 * j10);
        const double dxi = (j11 * rx - j01 * ry) * id;
        const double deta = (-j10 * rx + j00 * ry) * id;
        xi -= dxi;
        eta -= deta;
        if (fabs(dxi) + fabs(deta) < 1e-14) break;
    }
    l[0] = xi;
    l[1] = eta;
    l[2] = 0.0;
}

// computational gradients of the nine shape functions at local node `slot`:
// [dN/dX, dN/dY] = J^-T [dN/dxi, dN/deta], J the bilinear map's Jacobian there
__device__ __forceinline__ void q2_grad_at_node(const ElemRecQ &r, int slot, double gN[9][2])
{
    const double xs = double(q_xi(slot)), es = double(q_eta(slot));
    double Lx[3], dLx[3], Ly[3], dLy[3];
    lagrange3(xs, Lx, dLx);
    lagrange3(es, Ly, dLy);
    const Bilinear B = bilinear(r);
    const double j00 = B.b1.x + B.b3.x * es, j01 = B.b2.x + B.b3.x * xs;
    const double j10 = B.b1.y + B.b3.y * es, j11 = B.b2.y + B.b3.y * xs;
    const double id = rcp_nr(j00 * j11 - j01 * j10);
#pragma unroll
    for (int s = 0; s < 9; ++s) {
        const double dxi = dLx[q_xi(s) + 1] * Ly[q_eta(s) + 1];
        const double deta = Lx[q_xi(s) + 1] * dLy[q_eta(s) + 1];
        gN[s][0] = (j11 * dxi - j10 * deta) * id;
        gN[s][1] = (-j01 * dxi + j00 * deta) * id;
    }
}

// Walk over quadrilaterals.  The geometry is bilinear, so the edges are
// straight: P lies on the inner side of edge k when cross(c_{k+1} - c_k,
// P - c_k) >= 0, and in the element when all four hold to -TAU_LOC times
// twice the area (the quadrilateral's counterpart of a barycentric); else the
// walk crosses the edge with the most negative value (lowest edge on ties).
// Returns the element holding P (>= 0) with its node ids, or -1 wall, -2 far
// field, -4 cap; `last` is the last element visited inside the domain.
__device__ __forceinline__ int walk_rec_q(const ElemRecQ *__restrict__ el, double Lx, double Ly, int e,
                                          double &Px, double &Py, int nd[9], int &last)
{
    const bool periodic = Lx > 0.0 || Ly > 0.0;
    for (int it = 0; it < WALK_CAP; ++it) {
        const ElemRecQ &r = el[e];
        const double2 c[4] = {r.c[0], r.c[1], r.c[2], r.c[3]};
        const int4 nb = r.nb;
        const double a2 = r.a2;
        last = e;
        int k = 0;
        double mn = 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double2 p = c[j], q = c[(j + 1) & 3];
            const double v = (q.x - p.x) * (Py - p.y) - (q.y - p.y) * (Px - p.x);
            if (j == 0 || v < mn) {
                mn = v;
                k = j;
            }
        }
        if (mn >= -TAU_LOC * a2) {
            const int4 n03 = *reinterpret_cast<const int4 *>(&r.n[0]);
            const int4 n47 = *reinterpret_cast<const int4 *>(&r.n[4]);
            nd[0] = n03.x; nd[1] = n03.y; nd[2] = n03.z; nd[3] = n03.w;
            nd[4] = n47.x; nd[5] = n47.y; nd[6] = n47.z; nd[7] = n47.w;
            nd[8] = r.n[8];
            return e;
        }
        const int n = k == 0 ? nb.x : (k == 1 ? nb.y : (k == 2 ? nb.z : nb.w));
        if (n < 0) return n;
        if (periodic) {
            const int code = int((unsigned(r.codes) >> (4 * k)) & 15u);
            if (code != 4) {
                Px += double(code % 3 - 1) * Lx;
                Py += double(code / 3 - 1) * Ly;
            }
        }
        e = n;
    }
    return -4;
}

// ---- element kinds as template arguments of the kernels ----
struct EP2 {
    static constexpr int KIND = ELEM_P2;
    static constexpr int NV = 6;
    using Rec = ElemRec;
    using GRec = ElemGrad;  // what the node kernels read: gradient coefficients and node ids
    __device__ static const Rec *recs(const DevMesh &m) { return m.el; }
    __device__ static const GRec *grecs(const DevMesh &m) { return m.elg; }
    __device__ static void shape(const double l[3], double N[6]) { p2_shape(l, N); }
    template <typename T>
    __device__ static void grad_at_node(const T &r, int slot, double gN[6][2])
    {
        p2_grad_at_node(slot, r.a01, r.a23, gN);
    }
    // the three nodes of edge k: end, middle, end (counter-clockwise)
    __device__ static void edge_slots(int k, int s[3])
    {
        s[0] = (k + 1) % 3;
        s[1] = 3 + k;
        s[2] = (k + 2) % 3;
    }
};

struct EQ2 {
    static constexpr int KIND = ELEM_Q2;
    static constexpr int NV = 9;
    using Rec = ElemRecQ;
    using GRec = ElemRecQ;
    __device__ static const Rec *recs(const DevMesh &m) { return m.elq; }
    __device__ static const GRec *grecs(const DevMesh &m) { return m.elq; }
    __device__ static void shape(const double l[3], double N[9]) { q2_shape(l, N); }
    __device__ static void grad_at_node(const Rec &r, int slot, double gN[9][2]) { q2_grad_at_node(r, slot, gN); }
    __device__ static void edge_slots(int k, int s[3])
    {
        s[0] = k;
        s[1] = 4 + k;
        s[2] = (k + 1) & 3;
    }
};

// ---- equilibria, direction by direction (Sec. IV) ----
template <typename R>
__device__ __forceinline__ R phi1(int c, R u, R T)
{
    return c == 0 ? R(1) - (u * u + T) : (R(c) * u + u * u + T) * R(0.5);
}
template <typename R>
__device__ __forceinline__ R wc(int c, R T) { return c == 0 ? R(1) - T : T * R(0.5); }

template <typename R>
__device__ __forceinline__ R feq_i(int cx, int cy, R rho, R ux, R uy, R T)
{
    return rho * phi1(cx, ux, T) * phi1(cy, uy, T);
}

// general form G_i(M0, M_a, M_ab, Psi_i) of eq. geq_gstar
// (iT = 1/T and ih = 1/(2 T^2) are passed in so that a node's nine directions share them)
template <typename R>
__device__ __forceinline__ R gform_i(int cx, int cy, R T, R iT, R ih, R M0, R Mx, R My, R Mxx, R Mxy, R Myy,
                                     R psi)
{
    const R fx = R(cx), fy = R(cy);
    const R W = wc(cx, T) * wc(cy, T);
    const R quad = ((Mxx - M0 * T) * (fx * fx - T) + R(2) * Mxy * fx * fy + (Myy - M0 * T) * (fy * fy - T)) * ih;
    return W * (M0 + (Mx * fx + My * fy) * iT + quad) + psi;
}

// B_ia: 1 for the rest velocity, else -|c_ia - c_ia c_i^2 / 2|
template <typename R>
__device__ __forceinline__ R bcoef(int ca, int c2)
{
    return c2 == 0 ? R(1) : -fabs(R(ca) - R(0.5) * R(ca) * R(c2));
}

// parts of g^eq shared by all directions
template <typename R>
struct GeqParts {
    R M0, qx, qy, Rxx, Rxy, Ryy, Zx, Zy, iT, ih;
};

template <typename R>
__device__ __forceinline__ GeqParts<R> geq_parts(R rho, R ux, R uy, R T, R E)
{
    GeqParts<R> p;
    p.M0 = R(2) * rho * E;
    p.qx = R(2) * rho * ux * (E + T);
    p.qy = R(2) * rho * uy * (E + T);
    p.Rxx = R(2) * rho * E * (T + ux * ux) + R(2) * rho * T * (T + R(2) * ux * ux);
    p.Rxy = R(2) * rho * E * (ux * uy) + R(2) * rho * T * (R(2) * ux * uy);
    p.Ryy = R(2) * rho * E * (T + uy * uy) + R(2) * rho * T * (T + R(2) * uy * uy);
    p.iT = R(1) / T;
    p.ih = R(1) / (R(2) * T * T);
    p.Zx = rho * (R(1) - R(3) * T) * (T * T + R(2) * ux * ux * T + E * ux * ux) * p.iT;
    p.Zy = rho * (R(1) - R(3) * T) * (T * T + R(2) * uy * uy * T + E * uy * uy) * p.iT;
    return p;
}

template <typename R>
__device__ __forceinline__ R psi_i(int cx, int cy, const GeqParts<R> &p)
{
    const int c2 = cx * cx + cy * cy;
    return bcoef<R>(cx, c2) * p.Zx + bcoef<R>(cy, c2) * p.Zy;
}

__device__ __forceinline__ int xcd_block(int nblocks)
{
    // Workgroups are dealt round-robin over the 8 XCDs; give each XCD one
    // contiguous run of Hilbert-ordered tiles.  With nblocks = 8q + r, XCD x receives
    // q + (x < r) workgroups and its run starts at x q + min(x, r): a bijection
    // of [0, nblocks) for any nblocks.
    const int b = blockIdx.x;
    const int q = nblocks >> 3, r = nblocks & 7, x = b & 7;
    return x * q + min(x, r) + (b >> 3);
}

// The handle's error word, read past the caches (other workgroups of earlier
// kernels of the step, or of this one, may have raised it)
__device__ __forceinline__ int load_err(const int *err)
{
    return __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// a step kernel's workgroups return at once when an earlier step, or an
// earlier kernel of this one, has failed (one-wave workgroups, or kernels
// without block barriers: each wave decides for itself)
__device__ __forceinline__ bool wave_aborted(const int *err)
{
    return __builtin_amdgcn_readfirstlane(load_err(err)) != 0;
}
// the same decision for a whole multi-wave workgroup (before its first barrier)
__device__ __forceinline__ bool block_aborted(const int *err)
{
    __shared__ int s_abort;
    if (threadIdx.x == 0) s_abort = load_err(err);
    __syncthreads();
    return s_abort != 0;
}

// motion-law factors at one time level (shared by the clock, forces and move_mesh)
__device__ __forceinline__ MotionTime motion_time(const Motion &mo, double t)
{
    MotionTime tf{0, 0, 0, 0, 0, 0};
    if (mo.kind == 1) {
        sincos(2.0 * PI * t / mo.p[3], &tf.s, &tf.c);
    } else if (mo.kind == 2) {
        double s, c;
        sincos(mo.p[1] * t + mo.p[2], &s, &c);
        tf.yoff = -mo.p[0] * s;
        tf.vy = -mo.p[0] * mo.p[1] * c;
    } else if (mo.kind == 3) {
        const double A = mo.p[0], w = mo.p[1], php = mo.p[4], h = mo.p[5], phh = mo.p[6];
        double sp, cp, sh, ch;
        sincos(w * t + php, &sp, &cp);
        sincos(w * t + phh, &sh, &ch);
        sincos(A * sp, &tf.s, &tf.c);
        tf.thd = A * w * cp;
        tf.yoff = -h * sh;
        tf.vy = -h * w * ch;
        tf.iw = mo.p[8] > mo.p[7] ? 1.0 / (mo.p[8] - mo.p[7]) : 0.0;
    }
    return tf;
}

// case of the first node of a workgroup: every workgroup lies inside one case
__device__ __forceinline__ int block_case(const DevMesh &m, int first_node)
{
    return __builtin_amdgcn_readfirstlane(int(m.ncase[first_node]));
}

// R2: the (f_i, g_i) pair of one node, loaded and stored as one vector
template <typename R>
struct R2;
template <>
struct alignas(8) R2<float> {
    float x, y;
};
template <>
struct alignas(16) R2<double> {
    double x, y;
};

constexpr int SBLOCK = 64;  // k_stream: one wavefront per workgroup, no block barrier beyond the wave
// k_stream takes G groups of 7 nodes per workgroup (G = 1, 4, 8: the schedule's `groups`)
static_assert(CASE_ALIGN % (NODES_PER_WAVE * 8) == 0, "a k_stream workgroup must lie inside one case");
static_assert(NODES_PER_WAVE * 8 <= SBLOCK, "one lane per node in the metric phase");

// ---------------------------------------------------------------------------
// k_clock: per case, t -> t + dt; motion factors at t + dt/2 and t + dt.  It
// primes the clock after the host sets one; from then on each step's
// k_wall writes the next step's clock (the same arithmetic) into the other
// of the two clock buffers.
// ---------------------------------------------------------------------------
__device__ __forceinline__ CaseClock advance_clock(const CaseStatic &cs, double t, long long step)
{
    CaseClock k;
    const double dt = cs.ph.dt;
    k.th = motion_time(cs.mo, t + 0.5 * dt);
    k.t1 = motion_time(cs.mo, t + dt);
    k.t = t + dt;
    k.step = step + 1;
    return k;
}

__global__ void k_clock(const CaseStatic *__restrict__ cs, CaseClock *__restrict__ cc, int c0, int c1)
{
    const int c = c0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= c1) return;
    cc[c] = advance_clock(cs[c], cc[c].t, cc[c].step);
}

// ---------------------------------------------------------------------------
// Grad approximation at one node (Sec. IV.A, tab. Neq_Moments): targets and
// non-equilibrium moments, shared by the missing directions of the node
// ---------------------------------------------------------------------------
template <typename R>
struct GradTargets {
    R rho, ux, uy, T, E;
    R P1xx, P1xy, P1yy, q1x, q1y, R1xx, R1xy, R1yy;
    GeqParts<R> gp;
};

template <typename R, int MK, typename EK>
__device__ __forceinline__ GradTargets<R> grad_targets(const DevMesh &m, const R *__restrict__ mprev,
                                                        const Phys &ph, const Motion &mo, const MotionTime &t1,
                                                        int idx, double2 Xa, int e0, int slot)
{
    const double dt = ph.dt;
    double J1[4], v1[2];
    metric_k<MK>(mo, t1, Xa.x, Xa.y, J1, v1);
    GradTargets<R> g;
    const int w = m.wid[idx];
    if (w >= 0) {
        // wall node: wall velocity at t^{n+1}; rho and T of the previous step at B
        const int eb = m.bel[w];
        const double lb[3] = {m.blam[3 * w], m.blam[3 * w + 1], m.blam[3 * w + 2]};
        double Nb[EK::NV];
        EK::shape(lb, Nb);
        double rb = 0.0, Tb = 0.0;
        for (int s = 0; s < EK::NV; ++s) {
            const size_t nb = EK::grecs(m)[eb].n[s];
            rb += Nb[s] * double(mprev[4 * nb]);
            Tb += Nb[s] * double(mprev[4 * nb + 3]);
        }
        g.rho = R(rb);
        g.T = R(Tb);
        g.ux = R(v1[0]);
        g.uy = R(v1[1]);
    } else {
        // other node: its own values of the previous step
        g.rho = mprev[4 * size_t(idx)];
        g.ux = mprev[4 * size_t(idx) + 1];
        g.uy = mprev[4 * size_t(idx) + 2];
        g.T = mprev[4 * size_t(idx) + 3];
    }
    // gradients of the previous-step u and T at the node through the owner element
    const typename EK::GRec &r0 = EK::grecs(m)[e0];
    double gN[EK::NV][2];
    EK::grad_at_node(r0, slot, gN);
    double gr[3][2] = {{0, 0}, {0, 0}, {0, 0}};
    for (int s = 0; s < EK::NV; ++s) {
        const size_t nb = r0.n[s];
        const double u0 = double(mprev[4 * nb + 1]);
        const double u1 = double(mprev[4 * nb + 2]);
        const double tt = double(mprev[4 * nb + 3]);
        gr[0][0] += u0 * gN[s][0]; gr[0][1] += u0 * gN[s][1];
        gr[1][0] += u1 * gN[s][0]; gr[1][1] += u1 * gN[s][1];
        gr[2][0] += tt * gN[s][0]; gr[2][1] += tt * gN[s][1];
    }
    double dux_x, dux_y, duy_x, duy_y, dT_x, dT_y;
    to_physical(J1, gr[0][0], gr[0][1], dux_x, dux_y);
    to_physical(J1, gr[1][0], gr[1][1], duy_x, duy_y);
    to_physical(J1, gr[2][0], gr[2][1], dT_x, dT_y);
    const R Cv = R(ph.Cv), Cp = R(ph.Cp);
    g.E = Cv * g.T + R(0.5) * (g.ux * g.ux + g.uy * g.uy);
    const R om = R(1) / (R(ph.mu) / (g.rho * g.T * R(dt)) + R(0.5));
    const R om1 = R(1) / (R(ph.mu) / (R(ph.Pr) * g.rho * g.T * R(dt)) + R(0.5));
    const R dxux = R(dux_x), dyux = R(dux_y), dxuy = R(duy_x), dyuy = R(duy_y);
    const R Sxx = R(2) * dxux, Syy = R(2) * dyuy, Sxy = dxuy + dyux;
    const R divu = dxux + dyuy;
    const R dEx = Cv * R(dT_x) + g.ux * dxux + g.uy * dxuy;
    const R dEy = Cv * R(dT_y) + g.ux * dyux + g.uy * dyuy;
    const R pre = -(R(1) / om) * g.rho * g.T;
    g.P1xx = pre * (Sxx - divu / Cv);
    g.P1xy = pre * Sxy;
    g.P1yy = pre * (Syy - divu / Cv);
    const R pr1 = -(R(2) / om1) * g.rho * g.T;
    g.R1xx = pr1 * (Sxx * (g.E + R(2) * g.T) + g.ux * dEx + g.ux * dEx);
    g.R1xy = pr1 * (Sxy * (g.E + R(2) * g.T) + g.ux * dEy + g.uy * dEx);
    g.R1yy = pr1 * (Syy * (g.E + R(2) * g.T) + g.uy * dEy + g.uy * dEy);
    g.q1x = -(R(2) / om1) * g.rho * Cp * g.T * R(dT_x) + R(2) * (g.ux * g.P1xx + g.uy * g.P1xy);
    g.q1y = -(R(2) / om1) * g.rho * Cp * g.T * R(dT_y) + R(2) * (g.ux * g.P1xy + g.uy * g.P1yy);
    g.gp = geq_parts(g.rho, g.ux, g.uy, g.T, g.E);
    return g;
}

// f^miss = f^eq(targets) + dt f^(1), g^miss = g^eq(targets) + dt g^(1) for
// direction i, as deviations from the reference ref
template <typename R>
__device__ __forceinline__ void grad_missing(const GradTargets<R> &g, const R *__restrict__ ref, R dt, int i, R &fv,
                                             R &gv)
{
    const int cx = cx_of(i), cy = cy_of(i);
    const GeqParts<R> &gp = g.gp;
    const R f1 = gform_i(cx, cy, g.T, gp.iT, gp.ih, R(0), R(0), R(0), g.P1xx, g.P1xy, g.P1yy, R(0));
    const R g1 = gform_i(cx, cy, g.T, gp.iT, gp.ih, R(0), g.q1x, g.q1y, g.R1xx, g.R1xy, g.R1yy, R(0));
    fv = (feq_i(cx, cy, g.rho, g.ux, g.uy, g.T) - ref[2 * i]) + dt * f1;
    gv = (gform_i(cx, cy, g.T, gp.iT, gp.ih, gp.M0, gp.qx, gp.qy, gp.Rxx, gp.Rxy, gp.Ryy, psi_i(cx, cy, gp)) -
          ref[2 * i + 1]) + dt * g1;
}

// ---------------------------------------------------------------------------
// Streaming, one lane per (node, direction): the pieces shared by both
// streaming kernels.  Rows: metric (Sec. II), departure point (eq.
// Trasformed_Discrete_Vel, midpoint trace), walk (eq. NonLinear_Eq), P2 gather
// (eq. Propagation), missing populations (Sec. IV.A), moments (eq. Temp).
// ---------------------------------------------------------------------------

// departure point of direction (cx, cy) at a node X (P0 = X in the owner's
// frame): c^_i = J^-1 (c_i - v_g) at the node, then at the midpoint of the
// backward trajectory, both at t^{n+1/2}
// the node in the frame coded by `code` (periodic shift (sx+1) + 3 (sy+1)); on
// a non-periodic mesh the node itself
__device__ __forceinline__ void frame_origin(double2 Xa, int code, double Lx, double Ly, double &Px, double &Py)
{
    if (Lx > 0.0 || Ly > 0.0) {
        Px = Xa.x + double(code % 3 - 1) * Lx;
        Py = Xa.y + double(code / 3 - 1) * Ly;
    } else {
        Px = Xa.x;
        Py = Xa.y;
    }
}

// the node's part, shared by its nine directions: metric at the node and 1 / det J
template <int MK>
__device__ __forceinline__ void node_metric(const Motion &mo, const MotionTime &th, double2 Xa, int *err, int cur,
                                            double J[4], double v[2], double &id)
{
    metric_k<MK>(mo, th, Xa.x, Xa.y, J, v);
    const double det = J[0] * J[3] - J[1] * J[2];
    if (!(det > 0.0)) atomicOr(err, err_bits(ERR_JAC, cur));
    id = rcp_nr(det);
}

// the direction's part, from the node's metric (J0, v0, id0).  zone (blended
// pitch law only): 1 when the node's traces stay inside the rigid zone, where J
// at the midpoint is the node's rotation and the grid velocity the rigid
// branch's; 2 when they stay beyond the blend, where the mesh is at rest.
template <int MK>
__device__ __forceinline__ void departure_from(const Motion &mo, const MotionTime &th, double2 Xa, const double J0[4],
                                               const double v0[2], double id0, double P0x, double P0y, double dt,
                                               int cx, int cy, int *err, int cur, double &Px, double &Py,
                                               double &chx_out, double &chy_out, int zone = 0)
{
    double wx = double(cx) - v0[0], wy = double(cy) - v0[1];
    double chx = (J0[3] * wx - J0[1] * wy) * id0, chy = (-J0[2] * wx + J0[0] * wy) * id0;
    const double Xm = Xa.x - 0.5 * dt * chx, Ym = Xa.y - 0.5 * dt * chy;
    double J[4], v[2], id;
    if (MK == 3 && zone == 1) {
#pragma unroll
        for (int k = 0; k < 4; ++k) J[k] = J0[k];
        id = id0;
        const double rx = Xm - mo.p[2], ry = Ym - mo.p[3];
        v[0] = th.thd * (-th.s * rx - th.c * ry);
        v[1] = th.thd * (th.c * rx - th.s * ry) + th.vy;
    } else if (MK == 3 && zone == 2) {
        J[0] = 1.0; J[1] = 0.0; J[2] = 0.0; J[3] = 1.0;
        v[0] = 0.0; v[1] = 0.0;
        id = 1.0;
    } else {
        metric_k<MK>(mo, th, Xm, Ym, J, v);
        const double det = J[0] * J[3] - J[1] * J[2];
        if (!(det > 0.0)) atomicOr(err, err_bits(ERR_JAC, cur));
        id = rcp_nr(det);
    }
    wx = double(cx) - v[0];
    wy = double(cy) - v[1];
    chx = (J[3] * wx - J[1] * wy) * id;
    chy = (-J[2] * wx + J[0] * wy) * id;
    Px = P0x - dt * chx;
    Py = P0y - dt * chy;
    chx_out = chx;
    chy_out = chy;
}

// Interpolation of one (f_i, g_i) pair from the element's node values (6 or
// 9).  Since the weights sum to one, sum_s N_s f_s = f_0 + sum_{s>0} N_s (f_s - f_0): the
// rounded weights then multiply only differences, so in FP32 a uniform state
// is reproduced to one rounding and the weights' sum error does not drift the
// mass step after step.
template <typename R, int NV = 6>
__device__ __forceinline__ void p2_combine(const double Nd[NV], const R2<R> fg[NV], R &fv, R &gv)
{
    R dfv = 0, dgv = 0;
#pragma unroll
    for (int s = 1; s < NV; ++s) {
        dfv += R(Nd[s]) * (fg[s].x - fg[0].x);
        dgv += R(Nd[s]) * (fg[s].y - fg[0].y);
    }
    fv = fg[0].x + dfv;
    gv = fg[0].y + dgv;
}

// the reference of the stored populations of a case, in the storage precision
template <typename R>
__device__ __forceinline__ const R *pop_ref(const CaseStatic &cs);
template <>
__device__ __forceinline__ const float *pop_ref<float>(const CaseStatic &cs)
{
    return cs.ref32;
}
template <>
__device__ __forceinline__ const double *pop_ref<double>(const CaseStatic &cs)
{
    return cs.ref64;
}

// A direction whose departure point left the domain: across the far field it
// takes the free-stream equilibrium here; across a wall (or after a walk past
// its cap) it is left to k_wall (Grad approximation, Sec. IV.A).  Returns the
// direction's mask bit.
template <typename R>
__device__ __forceinline__ int fill_missing(const StepArgs<R> &a, const CaseStatic *__restrict__ cs, int c, int e,
                                            int i, R &fv, R &gv)
{
    if (e == -2) {
        fv = pop_ref<R>(cs[c])[REF_FAR + 2 * i];
        gv = pop_ref<R>(cs[c])[REF_FAR + 2 * i + 1];
        return 1 << (16 + i);
    }
    fv = 0;
    gv = 0;
    if (e == -4) atomicOr(a.s.err, err_bits(ERR_LOCATE, a.cur));
    return 1 << i;
}

// eq. Temp from the sums over directions of the stored deviations and the
// reference's sums: rho, u = j / rho, E = sum g / (2 rho), T = (E - u^2/2) / Cv,
// with correctly rounded divides, the arithmetic of the collision's moments.
// These are the moments the next step's wall targets and this step's
// correction passes read; in FP32 a reciprocal of rho or the rounded 1/Cv (0.4
// is not an FP32 number) biases them by a fixed fraction of an ulp every
// step, which accumulates where the flow lingers.
template <typename R>
__device__ __forceinline__ void moments_from_sums(const R *__restrict__ ref, R drho, R djx, R djy, R dsg, R Cv,
                                                  R *__restrict__ out)
{
    const R rho = ref[REF_RHO] + drho, jx = ref[REF_JX] + djx, jy = ref[REF_JY] + djy, sg = ref[REF_SG] + dsg;
    const R ux = jx / rho, uy = jy / rho;
    const R E = sg / (R(2) * rho);
    out[0] = rho;
    out[1] = ux;
    out[2] = uy;
    out[3] = (E - R(0.5) * (ux * ux + uy * uy)) / Cv;
}

// ---------------------------------------------------------------------------
// k_stream: one 64-wide wavefront per workgroup takes G groups of 7
// consecutive nodes.  First one lane per node reads the node's data and
// evaluates the metric at the node (the part of the departure trace its nine
// directions share) into LDS: with G > 1 the wave evaluates it for 7 G nodes
// at once instead of 7.  Then, group by group, the wave holds 7 nodes x 9
// directions (lane 63 idles), so the 9 walks and gathers of a node run in
// parallel.  Each lane starts its walk at the element its departure point was
// found in the step before (the hint), reads whole element records so that
// the gather needs no further lookup, and stores the element it ends in as
// the next step's hint.  The result does not depend on the start element.
// ---------------------------------------------------------------------------
template <typename R, int MK, typename EK, int G>
__global__ __launch_bounds__(SBLOCK) void k_stream(StepArgs<R> a, const CaseStatic *__restrict__ cs,
                                                   const CaseClock *__restrict__ cc)
{
    constexpr int STREAM_NODES = NODES_PER_WAVE * G;
    __shared__ R red[4][SBLOCK];
    __shared__ int msk[SBLOCK];
    __shared__ double2 sh_x[STREAM_NODES];
    __shared__ int sh_info[STREAM_NODES];
    __shared__ double sh_m[7][STREAM_NODES];  // J (4), v_g (2), 1 / det J at the node, t^{n+1/2}
    __shared__ R sh_sum[4][STREAM_NODES];     // per node: sum f, sum c_x f, sum c_y f, sum g
    __shared__ int sh_mask[STREAM_NODES];     // per node: missing-direction mask
    const DevMesh &m = a.m;
    if (wave_aborted(a.s.err)) return;
    const int lane = threadIdx.x;
    const int base = a.node0 + xcd_block(gridDim.x) * STREAM_NODES;
    const int c = block_case(m, base);
    const Phys &ph = cs[c].ph;
    if (lane < STREAM_NODES) {
        const int n = base + lane;
        const int info = m.oinfo[n];
        sh_info[lane] = info;
        if (!(info & PAD_NODE)) {
            const double2 Xa = m.X[n];
            sh_x[lane] = Xa;
            double J[4], v[2], id;
            node_metric<MK>(cs[c].mo, cc[c].th, Xa, a.s.err, a.cur, J, v, id);
            sh_m[0][lane] = J[0];
            sh_m[1][lane] = J[1];
            sh_m[2][lane] = J[2];
            sh_m[3][lane] = J[3];
            sh_m[4][lane] = v[0];
            sh_m[5][lane] = v[1];
            sh_m[6][lane] = id;
        }
    }
    __syncthreads();
    const bool periodic = ph.Lx > 0.0 || ph.Ly > 0.0;
    const double dt = ph.dt;
    // kept rolled: unrolled, the G groups' live ranges overlap and take the
    // kernel from 72 to 76 registers, one wave per SIMD fewer (7 -> 6)
#pragma unroll 1
    for (int grp = 0; grp < G; ++grp) {
        // The lane's direction and its (c_x, c_y), in int, R and double, are
        // loop-invariant.  Kept live across the loop they cost the FP64 kernel
        // the registers of one wave per SIMD (80 -> 72: 7 waves instead of 6),
        // so there an empty asm hides the lane index from hoisting and they
        // are recomputed per group.  In FP32 the same change (72 -> 64
        // registers, 8 waves) measured no faster, so it is left out.
        int ln = lane;
        if constexpr (sizeof(R) == 8) asm volatile("" : "+v"(ln));
        const int nl = ln / Q;
        const int i = ln - Q * nl;
        const bool lane_ok = ln < Q * NODES_PER_WAVE;
        const int cx = cx_of(i), cy = cy_of(i);
        const int t = NODES_PER_WAVE * grp + nl;  // node within the tile (< STREAM_NODES when lane_ok)
        const int idx = base + t;
        const bool active = lane_ok && !(sh_info[lane_ok ? t : 0] & PAD_NODE);
        R fv = 0, gv = 0;
        int mk = 0;
        if (active) {
            const int hint = a.s.hint[Q * size_t(idx) + i];
            const double2 Xa = sh_x[t];
            const int code0 = hint & 15;
            const double J0[4] = {sh_m[0][t], sh_m[1][t], sh_m[2][t], sh_m[3][t]};
            const double v0[2] = {sh_m[4][t], sh_m[5][t]};
            double P0x, P0y, Px, Py, chx, chy;
            frame_origin(Xa, code0, ph.Lx, ph.Ly, P0x, P0y);
            departure_from<MK>(cs[c].mo, cc[c].th, Xa, J0, v0, sh_m[6][t], P0x, P0y, dt, cx, cy, a.s.err, a.cur, Px,
                               Py, chx, chy);
            double l[3];
            int nd[EK::NV], last = hint >> 4;
            int e;
            if constexpr (EK::KIND == ELEM_P2) {
                e = walk_rec(m.el, ph.Lx, ph.Ly, hint >> 4, Px, Py, l, nd, last);
            } else {
                e = walk_rec_q(m.elq, ph.Lx, ph.Ly, hint >> 4, Px, Py, nd, last);
            }
            const int code = periodic ? frame_code(ph.Lx, ph.Ly, Xa, dt, chx, chy, Px, Py) : 4;
            if (e >= 0) {
                if constexpr (EK::KIND == ELEM_P2) {
                    if (periodic) reframe(m.el[e], ph.Lx, ph.Ly, Xa, dt, chx, chy, code, l);
                } else {
                    // the point in the final element's frame, formed from the node's
                    // canonical coordinates (path-independent), then its (xi, eta)
                    if (periodic) {
                        Px = (Xa.x + double(code % 3 - 1) * ph.Lx) - dt * chx;
                        Py = (Xa.y + double(code / 3 - 1) * ph.Ly) - dt * chy;
                    }
                    q2_local(m.elq[e], Px, Py, l);
                }
                double Nd[EK::NV];
                EK::shape(l, Nd);
                const R *__restrict__ fin = a.s.pop[a.cur];
                R2<R> fg[EK::NV];
#pragma unroll
                for (int s = 0; s < EK::NV; ++s)
                    fg[s] = *reinterpret_cast<const R2<R> *>(fin + NPOP * size_t(nd[s]) + 2 * i);
                p2_combine<R, EK::NV>(Nd, fg, fv, gv);
            } else {
                mk = fill_missing(a, cs, c, e, i, fv, gv);
            }
            // The next walk starts from the element reached, in the node's frame
            // there.  A frame code outside 0..8 (a departure point more than a
            // period away, or a walk stopped at its cap after many periodic
            // crossings) would spill into the element bits: the hint is then
            // left as it was.
            const int nh = ((e >= 0 ? e : last) << 4) | code;
            if (code >= 0 && code <= 8 && nh != hint) a.s.hint[Q * size_t(idx) + i] = nh;
            R2<R> out;
            out.x = fv;
            out.y = gv;
            *reinterpret_cast<R2<R> *>(a.s.ft + NPOP * size_t(idx) + 2 * i) = out;
        }
        red[0][lane] = fv;
        red[1][lane] = R(cx) * fv;
        red[2][lane] = R(cy) * fv;
        red[3][lane] = gv;
        msk[lane] = mk;
        __syncthreads();
        // lanes 0-3 of a node sum one quantity each over its nine directions
        // (in direction order, as node_moments does); lane 4 joins the masks
        if (active && i < 4) {
            const R *q = &red[i][lane - i];
            R sum = 0;
#pragma unroll
            for (int d = 0; d < Q; ++d) sum += q[d];
            sh_sum[i][t] = sum;
        } else if (active && i == 4) {
            int mm = 0;
#pragma unroll
            for (int d = 0; d < Q; ++d) mm |= msk[lane - 4 + d];
            sh_mask[t] = mm;
        }
        __syncthreads();  // red and msk are rewritten by the next group
    }
    // the tile's moments (eq. Temp), one lane per node; nodes with wall-crossing
    // directions go to k_wall's list instead
    if (lane < STREAM_NODES && !(sh_info[lane] & PAD_NODE)) {
        const int idx = base + lane;
        const int mm = sh_mask[lane];
        if (a.s.mask) a.s.mask[idx] = mm;
        if (mm & 0x1ff) {
            const int pos = atomicAdd(a.s.wcount, 1);
            if (pos < a.node1 - a.node0) a.s.wlist[pos] = make_int2(idx, mm & 0x1ff);
        } else {
            moments_from_sums(pop_ref<R>(cs[c]), sh_sum[0][lane], sh_sum[1][lane], sh_sum[2][lane],
                              sh_sum[3][lane], R(ph.Cv), a.s.mac[1 - a.cur] + 4 * size_t(idx));
        }
    }
}

constexpr int WALL_BLOCKS = 256;  // k_wall: smallest grid (grid-stride over the listed nodes)

// ---------------------------------------------------------------------------
// Collision arithmetic shared by the schedules (eqs. feqn, geqn, Ai).
//   f*_i = f'_i + dt A_ia X_a,   f'_i = f~_i + w (f^eq_i - f~_i),
//   g*_i = g~_i + w (g^eq_i - g~_i) + (w1 - w)(g^qe_i - g~_i).
// The one-wave schedules form f* in k_collide; the tile schedules store f'
// and add dt A_ia X_a when the next step stages the populations.  Both add
// it with add_phi, so the two give the same f* to the last bit.
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ R add_phi(R fp, R dt, R Ax, R Ay, R Xx, R Xy)
{
    return fma(dt, fma(Ay, Xy, Ax * Xx), fp);
}
// A_ia = c_ia - c_ia c_i^2 / 2 of direction i
template <typename R>
__device__ __forceinline__ R fold_phi(int i, R fp, R dt, R Xx, R Xy)
{
    const int cx = cx_of(i), cy = cy_of(i), c2 = cx * cx + cy * cy;
    const R Ax = R(cx) - R(0.5) * R(cx) * R(c2);
    const R Ay = R(cy) - R(0.5) * R(cy) * R(c2);
    return add_phi(fp, dt, Ax, Ay, Xx, Xy);
}

// One node's collision, in place on its 9 + 9 streamed populations: moments
// with correctly rounded divides (they set the equilibria every step, where
// the extra rounding of a reciprocal, and of 1 / Cv in FP32, would bias the
// FP32 path), equilibria, quasi-equilibrium, relaxation; with_x adds the
// correction dt A_ia X_a.  Returns true if a result is not finite.
template <typename R>
__device__ __forceinline__ bool relax(const Phys &ph, const R *__restrict__ ref, R f[Q], R g[Q], bool with_x, R Xx,
                                      R Xy)
{
    R rho = 0, jx = 0, jy = 0, pxx = 0, pxy = 0, pyy = 0, sg = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const R cx = R(CX_[i]), cy = R(CY_[i]);
        rho += f[i];
        jx += cx * f[i];
        jy += cy * f[i];
        pxx += cx * cx * f[i];
        pxy += cx * cy * f[i];
        pyy += cy * cy * f[i];
        sg += g[i];
    }
    rho += ref[REF_RHO];
    jx += ref[REF_JX];
    jy += ref[REF_JY];
    pxx += ref[REF_PXX];
    pxy += ref[REF_PXY];
    pyy += ref[REF_PYY];
    sg += ref[REF_SG];
    const R ux = jx / rho, uy = jy / rho;
    const R E = sg / (R(2) * rho);
    const R T = (E - R(0.5) * (ux * ux + uy * uy)) / R(ph.Cv);
    const R dt = R(ph.dt);
    const R om = R(1) / (R(ph.mu) / (rho * T * dt) + R(0.5));
    const R om1 = R(1) / (R(ph.mu) / (R(ph.Pr) * rho * T * dt) + R(0.5));
    const GeqParts<R> gp = geq_parts(rho, ux, uy, T, E);
    // q* = q^eq + 2 u_b (P_ab - P^eq_ab)
    const R dPxx = pxx - (rho * ux * ux + rho * T);
    const R dPxy = pxy - rho * ux * uy;
    const R dPyy = pyy - (rho * uy * uy + rho * T);
    const R qsx = gp.qx + R(2) * (ux * dPxx + uy * dPxy);
    const R qsy = gp.qy + R(2) * (ux * dPxy + uy * dPyy);
    // The moving directions relax towards their equilibria; the rest direction
    // takes minus the sum of their increments.  In exact arithmetic the two
    // agree (the equilibria carry the node's density and energy), but the
    // rounding of the equilibria is smooth in the moments: in a region of slow
    // flow it would add the same small amount of mass and energy at every step.
    bool bad = false;
    R sf = 0, sg1 = 0, sq = 0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const int cx = CX_[i], cy = CY_[i];
        const R ps = psi_i(cx, cy, gp);
        const R df = (feq_i(cx, cy, rho, ux, uy, T) - ref[2 * i]) - f[i];
        const R dg = (gform_i(cx, cy, T, gp.iT, gp.ih, gp.M0, gp.qx, gp.qy, gp.Rxx, gp.Rxy, gp.Ryy, ps) -
                      ref[2 * i + 1]) - g[i];
        const R dq = (gform_i(cx, cy, T, gp.iT, gp.ih, gp.M0, qsx, qsy, gp.Rxx, gp.Rxy, gp.Ryy, ps) -
                      ref[2 * i + 1]) - g[i];
        sf += df;
        sg1 += dg;
        sq += dq;
        R fo = fma(om, df, f[i]);
        if (with_x) fo = fold_phi(i, fo, dt, Xx, Xy);
        const R go = g[i] + om * dg + (om1 - om) * dq;
        f[i] = fo;
        g[i] = go;
        bad |= !isfinite(fo) || !isfinite(go);
    }
    {
        R fo = fma(om, -sf, f[0]);
        if (with_x) fo = fold_phi(0, fo, dt, Xx, Xy);
        const R go = g[0] - om * sg1 - (om1 - om) * sq;
        f[0] = fo;
        g[0] = go;
        bad |= !isfinite(fo) || !isfinite(go);
    }
    return bad;
}

// What the correction passes read at a node: the shape-function gradients of
// its owner element at the node's slot and the element's node ids; from the
// FP32-rounded copies when the state is FP32 (P2).
template <typename R, typename EK>
__device__ __forceinline__ void owner_gradient(const DevMesh &m, int idx, int info, double gN[EK::NV][2],
                                               int nd[EK::NV])
{
    const int e = m.own[idx];
    if constexpr (sizeof(R) == 4 && EK::KIND == ELEM_P2) {
        const ElemGradF &r = m.elgf[e];
        const float2 a01 = r.a01, a23 = r.a23;
        p2_grad_at_node(info_slot(info), make_double2(a01.x, a01.y), make_double2(a23.x, a23.y), gN);
#pragma unroll
        for (int s = 0; s < EK::NV; ++s) nd[s] = r.n[s];
    } else {
        const typename EK::GRec &r = EK::grecs(m)[e];
        EK::grad_at_node(r, info_slot(info), gN);
#pragma unroll
        for (int s = 0; s < EK::NV; ++s) nd[s] = r.n[s];
    }
}

// The point at which the correction passes evaluate J for a node: under the
// blended pitch law a node of the rigid zone takes the rotation centre and one
// beyond the blend a point beyond it (J is the same at every point of either
// zone, to the bit), so that only the nodes of the blend read their
// coordinates; these come from the FP32-rounded copy when the state is FP32 (P2).
template <typename R, int MK, typename EK>
__device__ __forceinline__ double2 jacobian_point(const DevMesh &m, const Motion &mo, int idx, int info)
{
    if constexpr (MK == 3) {
        if (info & INFO_RIGID) return make_double2(mo.p[2], mo.p[3]);
        if (info & INFO_REST) return make_double2(mo.p[2] + 2.0 * mo.p[8] + 1.0, mo.p[3]);
    }
    if constexpr (sizeof(R) == 4 && EK::KIND == ELEM_P2) {
        const float2 x = m.Xf[idx];
        return make_double2(x.x, x.y);
    } else {
        return m.X[idx];
    }
}

// X_a = -[g^-1 grad_X W_a]_a at node idx through its owner element, g^-1 = J^-T at t^{n+1}
template <typename R, int MK, typename EK>
__device__ __forceinline__ void correction_x(const DevMesh &m, const R *__restrict__ W, const Motion &mo,
                                             const MotionTime &t1, int idx, int info, R &Xx, R &Xy)
{
    double gN[EK::NV][2];
    int nd[EK::NV];
    owner_gradient<R, EK>(m, idx, info, gN, nd);
    const double2 Xa = jacobian_point<R, MK, EK>(m, mo, idx, info);
    double wxx = 0, wxy = 0, wyx = 0, wyy = 0;
#pragma unroll
    for (int s = 0; s < EK::NV; ++s) {
        const size_t nb = nd[s];
        const double w0 = double(W[2 * nb]), w1 = double(W[2 * nb + 1]);
        wxx += w0 * gN[s][0];
        wxy += w0 * gN[s][1];
        wyx += w1 * gN[s][0];
        wyy += w1 * gN[s][1];
    }
    double J[4], v[2];
    metric_k<MK>(mo, t1, Xa.x, Xa.y, J, v);
    double d0x, d0y, d1x, d1y;
    to_physical(J, wxx, wxy, d0x, d0y);
    to_physical(J, wyx, wyy, d1x, d1y);
    Xx = R(-d0x);
    Xy = R(-d1y);
}

// ---------------------------------------------------------------------------
// Tile kernel helpers
// ---------------------------------------------------------------------------
// walk in global memory from element e with at most `cap` steps: the element
// holding P (>= 0) with its barycentrics, or -1 wall, -2 far field, -4 cap
__device__ __forceinline__ int walk_capped(const ElemRec *__restrict__ el, double Lx, double Ly, int e, double &Px,
                                           double &Py, double l[3], int cap)
{
    for (int it = 0; it < cap; ++it) {
        const ElemRec &r = el[e];
        int k;
        if (walk_test(r.v0, r.a01, r.a23, Px, Py, l, k)) return e;
        e = walk_cross(Lx, Ly, r.nb, k, Px, Py);
        if (e < 0) return e;
    }
    return -4;
}

// (f*_i, g*_i) of node slot s: stored (f'_i, g*_i) with dt A_ia X_a added
template <typename R>
__device__ __forceinline__ R2<R> staged_pair(const R *__restrict__ fin, const R *__restrict__ xin, size_t s, int i,
                                             R dt)
{
    R2<R> v = *reinterpret_cast<const R2<R> *>(fin + NPOP * s + 2 * i);
    const R2<R> x = *reinterpret_cast<const R2<R> *>(xin + 2 * s);
    v.x = fold_phi(i, v.x, dt, x.x, x.y);
    return v;
}

template <typename R>
__host__ __device__ constexpr size_t tile_pop_bytes(int pn)
{
    return ((sizeof(R2<R>) * Q * size_t(pn)) + 15) & ~size_t(15);
}

// Dynamic LDS of the tile kernel.  Pointers into it are formed from this
// symbol where they are used, so that the compiler keeps them in the LDS
// address space (ds_read) instead of generic (flat) pointers.
extern __shared__ __align__(16) char tile_lds[];

// What one thread of the tile kernel needs for its node's directions; the
// case's constants are copies in registers, read once per workgroup.
template <typename R>
struct TileNode {
    Motion mo;
    MotionTime th;
    double dt, Lx, Ly;
    int pop_bytes;        // LDS bytes of the staged pairs: the element records follow
    int pem, pe0;         // pe_max; first patch element of the tile in the global tables
    bool staged;
    int e0;               // start of the walks off the patch: the owner element (global index)
    uint4 start;          // start of each direction's walk in the patch (local indices, 10 bits each)
    double2 Xa;
    double J0[4], v0[2], id0, P0x, P0y;
    int zone;             // departure_from's zone: 1 rigid, 2 at rest, 0 otherwise
};

// Walk over the patch staged in LDS from local element e (eq. NonLinear_Eq):
// the local element holding P, -1 wall, -2 far field, -4 cap; or, when it
// leaves the patch, the global element it goes on from (local = false).
__device__ __forceinline__ int tile_walk(const DevMesh &m, const TileArgs &ta, const double2 *rg, const uint4 *Le,
                                         int pem, int pe0, double Lx, double Ly, int e, double &Px, double &Py,
                                         double l[3], bool &local, int &steps)
{
    local = true;
    for (steps = 0; steps < WALK_CAP; ++steps) {
        int k;
        if (walk_test(rg[e], rg[pem + e], rg[2 * pem + e], Px, Py, l, k)) return e;
        const uint4 tp = Le[3 * pem + e];
        const unsigned nl = (tp.z >> (10 * k)) & 1023u;
        if (nl >= TL_OUT) {
            if (nl == TL_WALL) return -1;
            if (nl == TL_FAR) return -2;
            // the walk leaves the patch: on from the element across edge k
            local = false;
            ++steps;
            return walk_cross(Lx, Ly, m.el[ta.pelem[pe0 + e]].nb, k, Px, Py);
        }
        const int code = int((tp.w >> (4 * k)) & 15u);
        if (code != 4) {
            Px += double(code % 3 - 1) * Lx;
            Py += double(code / 3 - 1) * Ly;
        }
        e = int(nl);
    }
    return -4;
}

// Departure point, walk and P2 gather of direction i of a tile node (Sec. II
// eq. Trasformed_Discrete_Vel, Sec. III eqs. NonLinear_Eq and Propagation);
// the far-field and wall directions set their mask bits.
template <typename R, int MK>
__device__ __forceinline__ void tile_direction(const StepArgs<R> &a, const TileArgs &ta, const CaseStatic *cs,
                                               const CaseClock *cc, int c, const TileNode<R> &nd, int i, R &fv,
                                               R &gv, int &mw, int &mf)
{
    const DevMesh &m = a.m;
    const double dt = nd.dt, Lx = nd.Lx, Ly = nd.Ly;
    const bool periodic = Lx > 0.0 || Ly > 0.0;
    double Dx, Dy, chx, chy;  // the departure point, in the frame of the node's owner
    departure_from<MK>(nd.mo, nd.th, nd.Xa, nd.J0, nd.v0, nd.id0, nd.P0x, nd.P0y, dt, cx_of(i), cy_of(i), a.s.err,
                       a.cur, Dx, Dy, chx, chy, nd.zone);
    double l[3], Px = Dx, Py = Dy;
    int e, steps = 0;
    bool local = nd.staged;
    const R2<R> *Lp = reinterpret_cast<const R2<R> *>(tile_lds);
    const uint4 *Le = reinterpret_cast<const uint4 *>(tile_lds + nd.pop_bytes);
    const double2 *rg = reinterpret_cast<const double2 *>(tile_lds + nd.pop_bytes);
    const int pem = nd.pem;
    if (nd.staged) {
        const int owner = int(nd.start.w);
        const int e1 = int(((i < 3 ? nd.start.x : (i < 6 ? nd.start.y : nd.start.z)) >> (10 * (i % 3))) & 1023u);
        e = tile_walk(m, ta, rg, Le, pem, nd.pe0, Lx, Ly, e1, Px, Py, l, local, steps);
        if ((e == -1 || e == -2) && e1 != owner) {
            // a boundary decision is the walk's from the owner
            Px = Dx;
            Py = Dy;
            e = tile_walk(m, ta, rg, Le, pem, nd.pe0, Lx, Ly, owner, Px, Py, l, local, steps);
        }
    } else {
        e = nd.e0;
    }
    if (!local && e >= 0) e = walk_capped(m.el, Lx, Ly, e, Px, Py, l, WALK_CAP - steps);
    fv = 0;
    gv = 0;
    if (e >= 0) {
        if (periodic) {
            // the point again in the final element's frame, from the node's
            // canonical coordinates: the result does not depend on the path
            const int code = frame_code(Lx, Ly, nd.Xa, dt, chx, chy, Px, Py);
            const double Qx = (nd.Xa.x + double(code % 3 - 1) * Lx) - dt * chx;
            const double Qy = (nd.Xa.y + double(code / 3 - 1) * Ly) - dt * chy;
            if (local) {
                barycentric(rg[e], rg[pem + e], rg[2 * pem + e], Qx, Qy, l);
            } else {
                const ElemRec &r = m.el[e];
                barycentric(r.v0, r.a01, r.a23, Qx, Qy, l);
            }
        }
        double Nd[6];
        p2_shape(l, Nd);
        R2<R> fg[6];
        if (local) {
            const uint4 tp = Le[3 * pem + e];
#pragma unroll
            for (int s2 = 0; s2 < 6; ++s2) {
                const unsigned w = s2 < 3 ? tp.x : tp.y;
                fg[s2] = Lp[Q * ((w >> (10 * (s2 % 3))) & 1023u) + i];
            }
        } else {
            const int2 n01 = *reinterpret_cast<const int2 *>(&m.el[e].n[0]);
            const int2 n23 = *reinterpret_cast<const int2 *>(&m.el[e].n[2]);
            const int2 n45 = *reinterpret_cast<const int2 *>(&m.el[e].n[4]);
            const int nn[6] = {n01.x, n01.y, n23.x, n23.y, n45.x, n45.y};
            const R dtR = R(dt);
#pragma unroll
            for (int s2 = 0; s2 < 6; ++s2)
                fg[s2] = staged_pair(a.s.pop[a.cur], a.s.Xs[a.cur], size_t(nn[s2]), i, dtR);
        }
        p2_combine<R, 6>(Nd, fg, fv, gv);
    } else if (e == -2) {
        fv = pop_ref<R>(cs[c])[REF_FAR + 2 * i];  // rare: the free stream across the far field
        gv = pop_ref<R>(cs[c])[REF_FAR + 2 * i + 1];
        mf |= 1 << (16 + i);
    } else {
        if (e == -4) atomicOr(a.s.err, err_bits(ERR_LOCATE, a.cur));
        mw |= 1 << i;
    }
}

// directions [I0, I1) of a tile node, unrolled, into f[i - I0], g[i - I0]
template <typename R, int MK, int I0, int I1>
__device__ __forceinline__ void tile_directions(const StepArgs<R> &a, const TileArgs &ta, const CaseStatic *cs,
                                                const CaseClock *cc, int c, const TileNode<R> &nd, R f[Q], R g[Q],
                                                int &mw, int &mf)
{
#pragma unroll
    for (int i = I0; i < I1; ++i) tile_direction<R, MK>(a, ta, cs, cc, c, nd, i, f[i - I0], g[i - I0], mw, mf);
}
template <typename R, int I0, int I1>
__device__ __forceinline__ void tile_store(R2<R> *row, const R f[Q], const R g[Q])
{
#pragma unroll
    for (int i = I0; i < I1; ++i) row[i] = R2<R>{f[i - I0], g[i - I0]};
}

// ---------------------------------------------------------------------------
// k_tile: the tile schedules' streaming kernel over a tile of T consecutive
// (Hilbert-ordered) node slots, with DG groups of T threads: group d takes
// directions [9 d / DG, 9 (d + 1) / DG) of every node of the tile, so that a
// node's nine walks run in DG threads and a workgroup holds DG times the
// waves for the same LDS.
//   1. The workgroup stages its patch in LDS: the element records (geometry,
//      local node and neighbour indices) copied as they are stored, and the
//      (f*_i, g*_i) pairs of every patch node, f*_i = f'_i + dt A_ia X_a
//      formed on the way in (the tile's own nodes are the first T rows).
//   2. The metric at each node is evaluated once (by the last group, while
//      the others stage) and shared through LDS; then each thread, direction
//      by direction, forms the departure point (midpoint trace, Sec. II eq.
//      Trasformed_Discrete_Vel), walks from the start table's element over
//      the patch (eq. NonLinear_Eq; again from the owner if the walk ends at
//      a boundary, and on in global memory if it leaves the patch) and
//      gathers from LDS (eq. Propagation).
//   3. Once every gather is done, each thread writes its directions' streamed
//      pairs into its node's row; then the first group forms the moments (eq.
//      Temp, sums in direction order) and the part of the collision the
//      node's own moments fix (relax without X) in the row.  A node with
//      wall-crossing directions keeps its streamed populations and is listed
//      for k_wall, which fills, sums and relaxes it.
//   4. The tile's rows leave as coalesced 16-byte stores.
// A tile whose patch did not fit the LDS budget walks and gathers in global
// memory throughout.
// ---------------------------------------------------------------------------
// Registers are held to what 6 waves per SIMD allow in FP32 (80 VGPRs) and 4
// in FP64: two or more workgroups then share a CU with the LDS they need.
template <typename R>
constexpr int tile_waves_per_simd() { return sizeof(R) == 4 ? 6 : 4; }

template <typename R, int MK, int T, int DG>
__global__ __launch_bounds__(T * DG, tile_waves_per_simd<R>()) void k_tile(StepArgs<R> a,
                                                                           const CaseStatic *__restrict__ cs,
                                                                           const CaseClock *__restrict__ cc,
                                                                           TileArgs ta)
{
    constexpr int NT = T * DG;
    char *smem = tile_lds;
    __shared__ int s_mask[T];  // per node: wall directions in bits 0-8, far-field directions in bits 16-24
    const DevMesh &m = a.m;
    if (block_aborted(a.s.err)) return;
    const int t = threadIdx.x;
    const int tn = t % T;        // node of the tile
    const int dg = t / T;        // direction group (uniform over a wave: T is a multiple of 64)
    const int tile = a.node0 / T + xcd_block(gridDim.x);
    const int base = tile * T;
    const int c = block_case(m, base);
    const Phys &ph = cs[c].ph;
    const int4 hd = ta.hdr[tile];
    // LDS: the patch's (f*, g*) pairs [pn_max][9], then its element records as
    // four arrays [4][pe_max] of 16-byte words (v0, A01, A23, topology): lanes
    // reading nearby elements then read nearby words, not words 64 bytes apart
    // that share a few banks
    R2<R> *Lp = reinterpret_cast<R2<R> *>(smem);
    uint4 *Le = reinterpret_cast<uint4 *>(smem + tile_pop_bytes<R>(ta.pn_max));
    TileNode<R> nd;
    nd.mo = cs[c].mo;
    nd.th = cc[c].th;
    nd.dt = ph.dt;
    nd.Lx = ph.Lx;
    nd.Ly = ph.Ly;
    nd.pop_bytes = int(tile_pop_bytes<R>(ta.pn_max));
    nd.pem = ta.pe_max;
    nd.pe0 = hd.x;
    nd.staged = hd.y >= 0;
    const int n = base + tn;
    const int info = m.oinfo[n];
    const bool active = !(info & PAD_NODE);
    double *mt = reinterpret_cast<double *>(tile_lds + nd.pop_bytes + 64 * size_t(nd.pem));
    if (active) nd.Xa = m.X[n];
    nd.zone = (info & INFO_RIGID) ? 1 : ((info & INFO_REST) ? 2 : 0);
    if (DG > 1 && dg == DG - 1 && active) {
        // the metric at the node (Sec. II), once per node: with more than one
        // group the last one evaluates it, while the waves of the threads
        // below stage the patch, and leaves it in LDS for every group (SoA
        // [7][T] doubles after the element records)
        double J0[4], v0[2], id0;
        node_metric<MK>(nd.mo, nd.th, nd.Xa, a.s.err, a.cur, J0, v0, id0);
#pragma unroll
        for (int k = 0; k < 4; ++k) mt[k * T + tn] = J0[k];
        mt[4 * T + tn] = v0[0];
        mt[5 * T + tn] = v0[1];
        mt[6 * T + tn] = id0;
    }
    if (nd.staged) {
        const uint4 *__restrict__ src = ta.rec + 4 * size_t(hd.x);
        // one thread per patch element, its four words with independent
        // loads, from thread hd.w on (cyclically): the threads below stage
        // the patch nodes, so no thread waits on two rounds of loads
        for (int e = t - hd.w; e < hd.y; e += NT) {
            if (e < 0) continue;
            uint4 w[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) w[k] = src[4 * e + k];
#pragma unroll
            for (int k = 0; k < 4; ++k) Le[k * nd.pem + e] = w[k];
        }
        const int *__restrict__ pn = ta.pnode + hd.z;
        const R dtR = R(ph.dt);
        // one thread per patch node: its nine pairs and X are loaded together
        // (independent loads, one latency), folded and written to its row
        const R *__restrict__ fin = a.s.pop[a.cur];
        const R *__restrict__ xin = a.s.Xs[a.cur];
        for (int p = t; p < hd.w; p += NT) {
            const size_t sl = size_t(pn[p]);
            R2<R> v[Q];
#pragma unroll
            for (int i = 0; i < Q; ++i) v[i] = *reinterpret_cast<const R2<R> *>(fin + NPOP * sl + 2 * i);
            const R2<R> x = *reinterpret_cast<const R2<R> *>(xin + 2 * sl);
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                v[i].x = fold_phi(i, v[i].x, dtR, x.x, x.y);
                Lp[Q * p + i] = v[i];
            }
        }
    }
    if (dg == 0) {
        s_mask[tn] = 0;
    }
    if (DG == 1 && active) node_metric<MK>(nd.mo, nd.th, nd.Xa, a.s.err, a.cur, nd.J0, nd.v0, nd.id0);
    __syncthreads();
    R2<R> *row = Lp + Q * tn;
    int mw = 0, mf = 0;
    if (active) {
        frame_origin(nd.Xa, info_code(info), nd.Lx, nd.Ly, nd.P0x, nd.P0y);
        if (DG > 1) {
#pragma unroll
            for (int k = 0; k < 4; ++k) nd.J0[k] = mt[k * T + tn];
            nd.v0[0] = mt[4 * T + tn];
            nd.v0[1] = mt[5 * T + tn];
            nd.id0 = mt[6 * T + tn];
        }
        if (nd.staged)
            nd.start = ta.start[n];
        else
            nd.e0 = m.own[n];
    }
    // the thread's directions (dg is uniform over a wave; padding slots compute nothing)
    constexpr int B1 = DG == 1 ? 9 : (DG == 2 ? 5 : 3), B2 = DG == 3 ? 6 : 9;
    R fr[Q], gr[Q];
    if (active) {
        if (dg == 0)
            tile_directions<R, MK, 0, B1>(a, ta, cs, cc, c, nd, fr, gr, mw, mf);
        else if (dg == 1)
            tile_directions<R, MK, B1, B2>(a, ta, cs, cc, c, nd, fr, gr, mw, mf);
        else
            tile_directions<R, MK, B2, 9>(a, ta, cs, cc, c, nd, fr, gr, mw, mf);
    }
    __syncthreads();  // every gather of the tile is done: its own rows may be overwritten
    if (active) {
        if (dg == 0)
            tile_store<R, 0, B1>(row, fr, gr);
        else if (dg == 1)
            tile_store<R, B1, B2>(row, fr, gr);
        else
            tile_store<R, B2, 9>(row, fr, gr);
    }
    if (active && DG > 1) {
        if (mw | mf) atomicOr(&s_mask[tn], mw | mf);
    }
    __syncthreads();
    if (dg == 0) {
        if (DG > 1) {
            const int mk = s_mask[tn];
            mw = mk & 0xffff;
            mf = mk & ~0xffff;
        }
        R f[Q], g[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const R2<R> p = row[i];
            f[i] = active ? p.x : R(0);  // padding slots leave zeros
            g[i] = active ? p.y : R(0);
        }
        if (active) {
            if (a.s.mask) a.s.mask[n] = mw | mf;
            if (a.flags & 4) {
                // diagnostics: the streamed populations (wall directions filled by k_wall)
#pragma unroll
                for (int i = 0; i < Q; ++i) *reinterpret_cast<R2<R> *>(a.s.ft + NPOP * size_t(n) + 2 * i) = row[i];
            }
            if (mw) {
                // wall-crossing directions: k_wall fills them, forms the moments and relaxes
                const int pos = atomicAdd(a.s.wcount, 1);
                if (pos < a.node1 - a.node0) a.s.wlist[pos] = make_int2(n, mw);
            } else {
                // eq. Temp from the sums in direction order; moments as the one-wave kernel stores them
                R rho = 0, jx = 0, jy = 0, sg = 0;
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    rho += f[i];
                    jx += R(cx_of(i)) * f[i];
                    jy += R(cy_of(i)) * f[i];
                    sg += g[i];
                }
                moments_from_sums(pop_ref<R>(cs[c]), rho, jx, jy, sg, R(ph.Cv), a.s.mac[1 - a.cur] + 4 * size_t(n));
                if (!(a.flags & 1)) {
                    const bool bad = relax(ph, pop_ref<R>(cs[c]), f, g, false, R(0), R(0));
                    if ((a.flags & 2) && bad) atomicOr(a.s.err, err_bits(ERR_NONFINITE, a.cur));
                }
            }
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) row[i] = R2<R>{f[i], g[i]};
    }
    __syncthreads();
    {
        constexpr int NV16 = T * NPOP * int(sizeof(R)) / 16;
        const float4 *srcv = reinterpret_cast<const float4 *>(smem);
        float4 *__restrict__ dst = reinterpret_cast<float4 *>(a.s.pop[1 - a.cur] + NPOP * size_t(base));
        for (int k = t; k < NV16; k += NT) dst[k] = srcv[k];
    }
}

// ---------------------------------------------------------------------------
// k_wall: the listed nodes' wall-crossing directions by the Grad approximation
// (Sec. IV.A, tab. Neq_Moments), targets computed once per node, then the
// node's moments (eq. Temp) over all nine directions in direction order.
// ---------------------------------------------------------------------------
// SPLIT (tile schedules): the listed nodes' streamed populations sit in their
// output rows; after the fill and the moments they are relaxed there like
// every other node of the tile kernel (relax without X).
template <typename R, int MK, typename EK, bool SPLIT>
__global__ __launch_bounds__(64) void k_wall(StepArgs<R> a, const CaseStatic *__restrict__ cs,
                                             const CaseClock *__restrict__ cc)
{
    const DevMesh &m = a.m;
    if (wave_aborted(a.s.err)) return;
    if (blockIdx.x == 0) {
        // the next step's clock of this launch's cases: the step's kernels
        // read this step's (cc), the other buffer.  Here rather than in the
        // step's last kernel, whose occupancy the motion law's sin/cos would
        // set (93 VGPRs against 66 in k_grad2).
        for (int j = threadIdx.x; j < a.c1 - a.c0; j += blockDim.x)
            a.clock_next[a.c0 + j] = advance_clock(cs[a.c0 + j], cc[a.c0 + j].t, cc[a.c0 + j].step);
    }
    const int count = min(*a.s.wcount, a.node1 - a.node0);
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < count; j += gridDim.x * blockDim.x) {
        const int2 w = a.s.wlist[j];
        const int idx = w.x;
        const int c = m.ncase[idx];
        const Phys &ph = cs[c].ph;
        // the node's streamed pairs are loaded before the targets' chain of
        // dependent loads (owner, record, moments), so that their latency overlaps it
        R2<R> *ft = reinterpret_cast<R2<R> *>((SPLIT ? a.s.pop[1 - a.cur] : a.s.ft) + NPOP * size_t(idx));
        R2<R> pin[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) pin[q] = ft[q];
        const GradTargets<R> g = grad_targets<R, MK, EK>(m, a.s.mac[a.cur], ph, cs[c].mo, cc[c].t1, idx,
                                                         m.X[idx], m.own[idx], info_slot(m.oinfo[idx]));
        R rho = 0, jx = 0, jy = 0, sg = 0;
        R f[Q], gg[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int cx = cx_of(q), cy = cy_of(q);
            R2<R> p = pin[q];
            if ((w.y >> q) & 1) {
                grad_missing(g, pop_ref<R>(cs[c]), R(ph.dt), q, p.x, p.y);
                if (!SPLIT) ft[q] = p;
            }
            f[q] = p.x;
            gg[q] = p.y;
            rho += p.x;
            jx += R(cx) * p.x;
            jy += R(cy) * p.x;
            sg += p.y;
        }
        moments_from_sums(pop_ref<R>(cs[c]), rho, jx, jy, sg, R(ph.Cv), a.s.mac[1 - a.cur] + 4 * size_t(idx));
        if constexpr (SPLIT) {
            if (a.flags & 4) {
                R2<R> *d = reinterpret_cast<R2<R> *>(a.s.ft + NPOP * size_t(idx));
#pragma unroll
                for (int q = 0; q < Q; ++q) d[q] = R2<R>{f[q], gg[q]};
            }
            if (!(a.flags & 1)) {
                const bool bad = relax(ph, pop_ref<R>(cs[c]), f, gg, false, R(0), R(0));
                if ((a.flags & 2) && bad) atomicOr(a.s.err, err_bits(ERR_NONFINITE, a.cur));
            }
#pragma unroll
            for (int q = 0; q < Q; ++q) ft[q] = R2<R>{f[q], gg[q]};
        }
    }
}

// ---------------------------------------------------------------------------
// k_grad1: W_a = (mu / rho T) [g^-1 grad_X Q'_a]_a,  Q'_a = rho u_a (1 - 3T) - rho u_a^3
// ---------------------------------------------------------------------------
template <typename R, int MK, typename EK, int NB>
__global__ __launch_bounds__(NB) void k_grad1(StepArgs<R> a, const CaseStatic *__restrict__ cs,
                                              const CaseClock *__restrict__ cc)
{
    const DevMesh &m = a.m;
    if (wave_aborted(a.s.err)) return;
    const int b0 = a.node0 + xcd_block(gridDim.x) * NB;
    const int idx = b0 + threadIdx.x;
    const int c = block_case(m, b0);
    const int info = m.oinfo[idx];
    if (info & PAD_NODE) return;
    const R *__restrict__ mac = a.s.mac[1 - a.cur];
    double gN[EK::NV][2];
    int nd[EK::NV];
    owner_gradient<R, EK>(m, idx, info, gN, nd);
    const double2 Xa = jacobian_point<R, MK, EK>(m, cs[c].mo, idx, info);
    double gx0 = 0, gy0 = 0, gx1 = 0, gy1 = 0;
#pragma unroll
    for (int s = 0; s < EK::NV; ++s) {
        const size_t nb = nd[s];
        const R rho = mac[4 * nb], ux = mac[4 * nb + 1], uy = mac[4 * nb + 2], T = mac[4 * nb + 3];
        const R qx = rho * ux * (R(1) - R(3) * T) - rho * ux * ux * ux;
        const R qy = rho * uy * (R(1) - R(3) * T) - rho * uy * uy * uy;
        gx0 += double(qx) * gN[s][0];
        gy0 += double(qx) * gN[s][1];
        gx1 += double(qy) * gN[s][0];
        gy1 += double(qy) * gN[s][1];
    }
    double J[4], v[2];
    metric_k<MK>(cs[c].mo, cc[c].t1, Xa.x, Xa.y, J, v);
    double px, py, qx_, qy_;
    to_physical(J, gx0, gy0, px, py);
    to_physical(J, gx1, gy1, qx_, qy_);
    const R rho = mac[4 * size_t(idx)], T = mac[4 * size_t(idx) + 3];
    const R k = R(cs[c].ph.mu) / (rho * T);
    a.s.W[2 * size_t(idx)] = k * R(px);
    a.s.W[2 * size_t(idx) + 1] = k * R(qy_);
}

// one node's collision on its 18 streamed populations in LDS, in place
template <typename R, int MK, typename EK>
__device__ __forceinline__ void collide_node(const StepArgs<R> &a, const CaseStatic *__restrict__ cs,
                                             const CaseClock *__restrict__ cc, int c, int idx, int info,
                                             R *__restrict__ pf)
{
    R f[Q], g[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        f[i] = pf[2 * i];
        g[i] = pf[2 * i + 1];
    }
    R Xx, Xy;
    correction_x<R, MK, EK>(a.m, a.s.W, cs[c].mo, cc[c].t1, idx, info, Xx, Xy);
    if (a.flags & 4) {  // diagnostics (ALE_LB_F_KEEP_MASKS): keep X for ale_lb_get_correction
        a.s.Xc[2 * size_t(idx)] = Xx;
        a.s.Xc[2 * size_t(idx) + 1] = Xy;
    }
    const bool bad = relax(cs[c].ph, pop_ref<R>(cs[c]), f, g, true, Xx, Xy);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        pf[2 * i] = f[i];
        pf[2 * i + 1] = g[i];
    }
    if ((a.flags & 2) && bad) atomicOr(a.s.err, err_bits(ERR_NONFINITE, a.cur));
}

// ---------------------------------------------------------------------------
// k_collide: X_a = -[g^-1 grad_X W_a]_a, then eqs. feqn / geqn
// ---------------------------------------------------------------------------
template <typename R, int MK, typename EK, int NB>
__global__ __launch_bounds__(NB) void k_collide(StepArgs<R> a, const CaseStatic *__restrict__ cs,
                                                const CaseClock *__restrict__ cc)
{
    // The workgroup's streamed populations (NB nodes x 18, contiguous) come in
    // through LDS with coalesced 16-byte loads, and the collided ones leave the
    // same way: read and written by one thread per node, every load and store
    // of a wave would touch 64 addresses 18 scalars apart.
    constexpr int NV16 = NB * NPOP * int(sizeof(R)) / 16;
    __shared__ float4 stage[NV16];
    const DevMesh &m = a.m;
    if (block_aborted(a.s.err)) return;
    const int b0 = a.node0 + xcd_block(gridDim.x) * NB;
    const int idx = b0 + threadIdx.x;
    const int c = block_case(m, b0);
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.s.wcount = 0;  // k_wall of this step has run
    {
        const float4 *__restrict__ src = reinterpret_cast<const float4 *>(a.s.ft + NPOP * size_t(b0));
        for (int k = threadIdx.x; k < NV16; k += NB) stage[k] = src[k];
    }
    __syncthreads();
    const int info = m.oinfo[idx];
    // no collision (tests) or a padding slot: the staged values leave unchanged
    if (!(info & PAD_NODE) && !(a.flags & 1))
        collide_node<R, MK, EK>(a, cs, cc, c, idx, info, reinterpret_cast<R *>(stage) + NPOP * threadIdx.x);
    __syncthreads();
    {
        float4 *__restrict__ dst = reinterpret_cast<float4 *>(a.s.pop[1 - a.cur] + NPOP * size_t(b0));
        for (int k = threadIdx.x; k < NV16; k += NB) dst[k] = stage[k];
    }
}


// ---------------------------------------------------------------------------
// k_grad2 (tile schedules): X_a = -[g^-1 grad_X W_a]_a into Xs[1 - cur], the
// correction the next step adds to f' as it stages the populations.
// ---------------------------------------------------------------------------
template <typename R, int MK, typename EK, int NB>
__global__ __launch_bounds__(NB) void k_grad2(StepArgs<R> a, const CaseStatic *__restrict__ cs,
                                              const CaseClock *__restrict__ cc)
{
    const DevMesh &m = a.m;
    if (wave_aborted(a.s.err)) return;
    const int b0 = a.node0 + xcd_block(gridDim.x) * NB;
    const int idx = b0 + threadIdx.x;
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.s.wcount = 0;  // k_wall of this step has run
    const int info = m.oinfo[idx];
    R Xx = 0, Xy = 0;
    if (!(info & PAD_NODE) && !(a.flags & 1)) {
        const int c = block_case(m, b0);
        correction_x<R, MK, EK>(m, a.s.W, cs[c].mo, cc[c].t1, idx, info, Xx, Xy);
        // part of the step's post-collision state: checked like the populations
        if ((a.flags & 2) && !(isfinite(Xx) && isfinite(Xy))) atomicOr(a.s.err, err_bits(ERR_NONFINITE, a.cur));
    }
    *reinterpret_cast<R2<R> *>(a.s.Xs[1 - a.cur] + 2 * size_t(idx)) = R2<R>{Xx, Xy};
}

// tile state -> post-collision state: f_i = f'_i + dt A_ia X_a in place, X cleared
template <typename R>
__global__ __launch_bounds__(BLOCK) void k_fold_x(DevMesh m, R *pop, R *X, const CaseStatic *cs)
{
    const int idx = blockIdx.x * BLOCK + threadIdx.x;
    if (idx >= m.N) return;
    const R dt = R(cs[m.ncase[idx]].ph.dt);
    R *p = pop + NPOP * size_t(idx);
    const R Xx = X[2 * size_t(idx)], Xy = X[2 * size_t(idx) + 1];
#pragma unroll
    for (int i = 0; i < Q; ++i) p[2 * i] = fold_phi(i, p[2 * i], dt, Xx, Xy);
    X[2 * size_t(idx)] = R(0);
    X[2 * size_t(idx) + 1] = R(0);
}

// free-stream equilibrium populations of every case (the far field's missing
// populations), and from them the reference of the stored populations in
// each precision: the equilibrium on the grid of the precision (2^-20 for
// FP32, 2^-44 for FP64), whose sums over directions are then exact in FP64
// and in the storage precision (values below 16 with at most 24, or 48,
// significant bits)
__global__ void k_freestream(CaseStatic *cs, int ncases)
{
    const int c = blockIdx.x;
    const int i = threadIdx.x;
    if (c >= ncases) return;
    CaseStatic &k = cs[c];
    if (i < Q) {
        const Phys &ph = k.ph;
        const double ri = ph.rho_inf, ux = ph.ux_inf, uy = ph.uy_inf, Ti = ph.T_inf;
        const double Ei = ph.Cv * Ti + 0.5 * (ux * ux + uy * uy);
        const GeqParts<double> gp = geq_parts(ri, ux, uy, Ti, Ei);
        const int cx = cx_of(i), cy = cy_of(i);
        k.finf[2 * i] = feq_i(cx, cy, ri, ux, uy, Ti);
        k.finf[2 * i + 1] = gform_i(cx, cy, Ti, gp.iT, gp.ih, gp.M0, gp.qx, gp.qy, gp.Rxx, gp.Rxy, gp.Ryy,
                                    psi_i(cx, cy, gp));
    }
    __syncthreads();
    if (i != 0) return;
    double s32[REF_FAR - NPOP] = {}, s64[REF_FAR - NPOP] = {};
    for (int q = 0; q < NPOP; ++q) {
        const double v = k.finf[q];
        const double r32 = ldexp(rint(ldexp(v, 20)), -20), r64 = ldexp(rint(ldexp(v, 44)), -44);
        k.ref32[q] = float(r32);
        k.ref64[q] = r64;
        k.ref32[REF_FAR + q] = float(v - r32);
        k.ref64[REF_FAR + q] = v - r64;
        const int d = q >> 1;
        const double cx = cx_of(d), cy = cy_of(d);
        const double wt[REF_SG - NPOP + 1] = {1.0, cx, cy, cx * cx, cx * cy, cy * cy, 0.0};  // rho, j, P, -
        for (int j = 0; j <= REF_SG - NPOP; ++j) {
            const double w = (q & 1) ? (j == REF_SG - NPOP ? 1.0 : 0.0) : wt[j];
            s32[j] += w * r32;
            s64[j] += w * r64;
        }
    }
    for (int j = 0; j < REF_FAR - NPOP; ++j) {
        k.ref32[NPOP + j] = float(s32[j]);
        k.ref64[NPOP + j] = s64[j];
    }
}

// ---------------------------------------------------------------------------
// initial condition: f = f^eq, g = g^eq (FP64 fields in internal order), stored
// as deviations from the reference
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(BLOCK) void k_init(DevMesh m, DevState<R> s, const CaseStatic *cs, const double *rho,
                                                const double *ux, const double *uy, const double *T, int cur)
{
    const int idx = blockIdx.x * BLOCK + threadIdx.x;
    if (idx >= m.N || (m.oinfo[idx] & PAD_NODE)) return;
    const CaseStatic &cc = cs[m.ncase[idx]];
    const R Cv = R(cc.ph.Cv);
    const R *__restrict__ ref = pop_ref<R>(cc);
    const R r = R(rho[idx]), u = R(ux[idx]), w = R(uy[idx]), t = R(T[idx]);
    const R E = Cv * t + R(0.5) * (u * u + w * w);
    const GeqParts<R> gp = geq_parts(r, u, w, t, E);
    R *p = s.pop[cur] + NPOP * size_t(idx);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int cx = CX_[i], cy = CY_[i];
        p[2 * i] = feq_i(cx, cy, r, u, w, t) - ref[2 * i];
        p[2 * i + 1] = gform_i(cx, cy, t, gp.iT, gp.ih, gp.M0, gp.qx, gp.qy, gp.Rxx, gp.Rxy, gp.Ryy,
                               psi_i(cx, cy, gp)) - ref[2 * i + 1];
    }
    R *mc = s.mac[cur] + 4 * size_t(idx);
    mc[0] = r;
    mc[1] = u;
    mc[2] = w;
    mc[3] = t;
}

__global__ __launch_bounds__(BLOCK) void k_move_mesh(DevMesh m, const CaseStatic *cs, const double *t_case,
                                                     double *x, double *Jinv, double *det, double *vg, int *err)
{
    const int idx = blockIdx.x * BLOCK + threadIdx.x;
    if (idx >= m.N || (m.oinfo[idx] & PAD_NODE)) return;
    const int c = m.ncase[idx];
    const Motion &mo = cs[c].mo;
    const MotionTime tf = motion_time(mo, t_case[c]);
    const double2 Xa = m.X[idx];
    double J[4], v[2], px, py;
    metric(mo, tf, Xa.x, Xa.y, J, v);
    position(mo, tf, Xa.x, Xa.y, px, py);
    const double d = J[0] * J[3] - J[1] * J[2];
    if (!(d > 0.0)) atomicOr(err, ERR_JAC);
    if (x) { x[2 * idx] = px; x[2 * idx + 1] = py; }
    if (Jinv) {
        Jinv[4 * idx] = J[3] / d;
        Jinv[4 * idx + 1] = -J[1] / d;
        Jinv[4 * idx + 2] = -J[2] / d;
        Jinv[4 * idx + 3] = J[0] / d;
    }
    if (det) det[idx] = d;
    if (vg) { vg[2 * idx] = v[0]; vg[2 * idx + 1] = v[1]; }
}

// ---------------------------------------------------------------------------
// forces: traction on straight wall edges (3 nodes each), Simpson weights 1/6 4/6 1/6,
// p = rho T, tau = mu (S - (1/Cv) div u I), gradients from the edge's element.
// Each workgroup sums the wall edges of one case in a fixed order; one thread
// per case then sums its workgroups' partials.
// ---------------------------------------------------------------------------
template <typename R, typename EK>
__global__ __launch_bounds__(BLOCK) void k_forces(DevMesh m, const R *mac, const CaseStatic *cs,
                                                  const CaseClock *cc, double *partial)
{
    __shared__ double red[6][BLOCK];
    const int4 fb = m.fblk[blockIdx.x];
    const int c = fb.x;
    const int w = fb.y + threadIdx.x;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    if (w < fb.z) {
        const Phys &ph = cs[c].ph;
        const Motion &mo = cs[c].mo;
        const MotionTime tf = motion_time(mo, cc[c].t);
        const int2 we = m.wedge[w];
        const int e = we.x, k = we.y;
        const typename EK::GRec &r = EK::grecs(m)[e];
        const double4 ab = m.wxy[w];
        double xa, ya, xb, yb;
        position(mo, tf, ab.x, ab.y, xa, ya);
        position(mo, tf, ab.z, ab.w, xb, yb);
        const double dx = xb - xa, dy = yb - ya;
        const double len = sqrt(dx * dx + dy * dy);
        const double nx = -dy / len, ny = dx / len;
        int slots[3];
        EK::edge_slots(k, slots);
        const double wts[3] = {1.0 / 6.0, 4.0 / 6.0, 1.0 / 6.0};
        for (int j = 0; j < 3; ++j) {
            const int s = slots[j];
            double gN[EK::NV][2];
            EK::grad_at_node(r, s, gN);
            const double X0 = j == 0 ? ab.x : (j == 2 ? ab.z : 0.5 * (ab.x + ab.z));
            const double Y0 = j == 0 ? ab.y : (j == 2 ? ab.w : 0.5 * (ab.y + ab.w));
            double gu[2][2] = {{0, 0}, {0, 0}};
            for (int q = 0; q < EK::NV; ++q) {
                const size_t nb = r.n[q];
                const double u0 = double(mac[4 * nb + 1]), u1 = double(mac[4 * nb + 2]);
                gu[0][0] += u0 * gN[q][0]; gu[0][1] += u0 * gN[q][1];
                gu[1][0] += u1 * gN[q][0]; gu[1][1] += u1 * gN[q][1];
            }
            double J[4], v[2];
            metric(mo, tf, X0, Y0, J, v);
            double G[2][2];
            to_physical(J, gu[0][0], gu[0][1], G[0][0], G[0][1]);
            to_physical(J, gu[1][0], gu[1][1], G[1][0], G[1][1]);
            const double divu = G[0][0] + G[1][1];
            double tau[2][2];
            for (int cc2 = 0; cc2 < 2; ++cc2)
                for (int d = 0; d < 2; ++d)
                    tau[cc2][d] = ph.mu * (G[cc2][d] + G[d][cc2] - (cc2 == d ? divu / ph.Cv : 0.0));
            const size_t an = r.n[s];
            const double pr = double(mac[4 * an]) * double(mac[4 * an + 3]);
            double xn, yn;
            position(mo, tf, X0, Y0, xn, yn);
            const double rx = xn - ph.refx, ry = yn - ph.refy;
            const double tpx = -pr * nx, tpy = -pr * ny;
            const double tvx = tau[0][0] * nx + tau[0][1] * ny, tvy = tau[1][0] * nx + tau[1][1] * ny;
            const double wl = wts[j] * len;
            acc[0] += wl * tpx;
            acc[1] += wl * tpy;
            acc[2] += wl * tvx;
            acc[3] += wl * tvy;
            acc[4] += -wl * (rx * tpy - ry * tpx);
            acc[5] += -wl * (rx * tvy - ry * tvx);
        }
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) red[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int half = BLOCK / 2; half > 0; half >>= 1) {
        if (threadIdx.x < half)
#pragma unroll
            for (int q = 0; q < 6; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + half];
        __syncthreads();
    }
    if (threadIdx.x < 6) partial[6 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void k_sum_partials(const double *partial, const int2 *case_blocks, int ncases, double *out)
{
    const int c = blockIdx.x;
    const int q = threadIdx.x;
    if (c >= ncases || q >= 6) return;
    double s = 0.0;
    for (int b = case_blocks[c].x; b < case_blocks[c].y; ++b) s += partial[6 * b + q];
    out[6 * c + q] = s;
}

// populations are stored f_0 g_0 f_1 g_1 ...; the FP64 side lists f_0..f_8 then g_0..g_8
__device__ __forceinline__ size_t host_component(size_t c, int C)
{
    return C == NPOP ? (c & 1) * Q + (c >> 1) : c;
}
template <typename R>
__global__ void k_convert(const R *src, double *dst, size_t n, int C, const R *X, const uint8_t *ncase,
                          const CaseStatic *cs)
{
    const size_t k = size_t(blockIdx.x) * BLOCK + threadIdx.x;
    if (k >= n * C) return;
    const size_t a = k / C, c = k - a * C;
    R v = src[k];
    double ref = 0.0;  // populations: the reference, added in FP64 (exact for FP32 storage)
    if (ncase) {
        const CaseStatic &cc = cs[ncase[a]];
        if (X && !(c & 1)) v = fold_phi(int(c >> 1), v, R(cc.ph.dt), X[2 * a], X[2 * a + 1]);
        ref = double(pop_ref<R>(cc)[c]);
    }
    dst[host_component(c, C) * n + a] = double(v) + ref;
}
template <typename R>
__global__ void k_convert_back(const double *src, R *dst, size_t n, int C, const uint8_t *ncase,
                               const CaseStatic *cs)
{
    const size_t k = size_t(blockIdx.x) * BLOCK + threadIdx.x;
    if (k >= n * C) return;
    const size_t a = k / C, c = k - a * C;
    const double ref = ncase ? double(pop_ref<R>(cs[ncase[a]])[c]) : 0.0;
    dst[k] = R(src[host_component(c, C) * n + a] - ref);
}

inline unsigned blocks_for(size_t n) { return unsigned((n + BLOCK - 1) / BLOCK); }

}  // namespace

// dynamic LDS of a tile workgroup: the patch's populations, then its element
// records, then the metric of the tile's T nodes (8 doubles each)
size_t tile_lds_bytes(int pe_max, int pn_max, int pop_bytes, int T)
{
    const size_t pop = pop_bytes == 4 ? tile_pop_bytes<float>(pn_max) : tile_pop_bytes<double>(pn_max);
    return pop + 64 * size_t(pe_max) + TILE_METRIC_BYTES * size_t(T);
}

template <typename R, int MK, typename EK>
hipError_t launch_one_wave(const StepArgs<R> &a, const CaseStatic *cs, const CaseClock *cc, int groups,
                           hipStream_t st)
{
    const int N = a.node1 - a.node0;
    switch (groups) {
    case 1:
        hipLaunchKernelGGL((k_stream<R, MK, EK, 1>), dim3(N / NODES_PER_WAVE), dim3(SBLOCK), 0, st, a, cs, cc);
        return hipSuccess;
    case 4:
        hipLaunchKernelGGL((k_stream<R, MK, EK, 4>), dim3(N / (4 * NODES_PER_WAVE)), dim3(SBLOCK), 0, st, a, cs,
                           cc);
        return hipSuccess;
    case 8:
        hipLaunchKernelGGL((k_stream<R, MK, EK, 8>), dim3(N / (8 * NODES_PER_WAVE)), dim3(SBLOCK), 0, st, a, cs,
                           cc);
        return hipSuccess;
    default: return hipErrorInvalidValue;
    }
}

template <typename R, int MK>
hipError_t launch_stream_k(const StepArgs<R> &a, const CaseStatic *cs, const CaseClock *cc, const Schedule &sch,
                           const TileArgs *ta, hipStream_t st)
{
    const int N = a.node1 - a.node0;
    if (a.m.kind == ELEM_Q2) {
        // quadrilateral meshes: the one-wave streaming kernel only
        if (sch.waves != 0) return hipErrorInvalidValue;
        return launch_one_wave<R, MK, EQ2>(a, cs, cc, sch.groups, st);
    }
    if (sch.waves == 0) return launch_one_wave<R, MK, EP2>(a, cs, cc, sch.groups, st);
    if (!ta || ta->tile != 64 * sch.waves) return hipErrorInvalidValue;
    const size_t lds = tile_lds_bytes(ta->pe_max, ta->pn_max, sizeof(R), ta->tile);
#define ALELB_TILE(T, DG) \
    hipLaunchKernelGGL((k_tile<R, MK, T, DG>), dim3(N / T), dim3(T * DG), lds, st, a, cs, cc, *ta)
    switch (sch.waves * 4 + sch.groups) {
    case 2 * 4 + 1: ALELB_TILE(128, 1); break;
    case 2 * 4 + 2: ALELB_TILE(128, 2); break;
    case 2 * 4 + 3: ALELB_TILE(128, 3); break;
    case 4 * 4 + 1: ALELB_TILE(256, 1); break;
    case 4 * 4 + 2: ALELB_TILE(256, 2); break;
    case 4 * 4 + 3: ALELB_TILE(256, 3); break;
    default: return hipErrorInvalidValue;
    }
#undef ALELB_TILE
    return hipSuccess;
}

// the correction passes: k_grad1, then k_collide (one-wave schedules) or k_grad2 (tile schedules)
template <typename R, int MK, typename EK, int NB>
hipError_t launch_nodes_nb(const StepArgs<R> &a, const CaseStatic *cs, const CaseClock *cc, bool tile,
                           hipStream_t st, hipEvent_t evmid)
{
    const int N = a.node1 - a.node0;
    hipError_t e = hipSuccess;
    if (!(a.flags & 1)) hipLaunchKernelGGL((k_grad1<R, MK, EK, NB>), dim3(N / NB), dim3(NB), 0, st, a, cs, cc);
    if (evmid && (e = hipEventRecord(evmid, st)) != hipSuccess) return e;
    if (!tile) {
        hipLaunchKernelGGL((k_collide<R, MK, EK, NB>), dim3(N / NB), dim3(NB), 0, st, a, cs, cc);
        return hipSuccess;
    }
    if constexpr (EK::KIND == ELEM_P2) {
        hipLaunchKernelGGL((k_grad2<R, MK, EK, NB>), dim3(N / NB), dim3(NB), 0, st, a, cs, cc);
        return hipSuccess;
    }
    return hipErrorInvalidValue;  // quadrilaterals have no tile schedule
}

template <typename R, int MK, typename EK>
hipError_t launch_nodes_ek(const StepArgs<R> &a, const CaseStatic *cs, const CaseClock *cc, const Schedule &sch,
                           hipStream_t st, hipEvent_t evmid)
{
    const bool tile = tiled(sch);
    switch (sch.node_block) {
    case 64: return launch_nodes_nb<R, MK, EK, 64>(a, cs, cc, tile, st, evmid);
    case 128: return launch_nodes_nb<R, MK, EK, 128>(a, cs, cc, tile, st, evmid);
    case 256: return launch_nodes_nb<R, MK, EK, 256>(a, cs, cc, tile, st, evmid);
    default: return hipErrorInvalidValue;
    }
}

template <typename R, int MK>
hipError_t launch_nodes_k(const StepArgs<R> &a, const CaseStatic *cs, const CaseClock *cc, const Schedule &sch,
                          hipStream_t st, hipEvent_t evmid)
{
    if (a.m.kind == ELEM_Q2) return launch_nodes_ek<R, MK, EQ2>(a, cs, cc, sch, st, evmid);
    return launch_nodes_ek<R, MK, EP2>(a, cs, cc, sch, st, evmid);
}

template <typename R, int MK>
hipError_t launch_wall_k(const StepArgs<R> &a, const CaseStatic *cs, const CaseClock *cc, const Schedule &sch,
                         hipStream_t st)
{
    // The list is filled on the device, so its length is unknown here; it is
    // mostly the wall nodes themselves.  A thread per two wall nodes keeps the
    // latency-bound per-node chain to about one pass per thread; the
    // grid-stride loop covers any longer list.
    const int nb = std::min(65535, std::max(WALL_BLOCKS, (2 * a.m.NW + 63) / 64));
    if (a.m.kind == ELEM_Q2)
        hipLaunchKernelGGL((k_wall<R, MK, EQ2, false>), dim3(nb), dim3(64), 0, st, a, cs, cc);
    else if (tiled(sch))
        hipLaunchKernelGGL((k_wall<R, MK, EP2, true>), dim3(nb), dim3(64), 0, st, a, cs, cc);
    else
        hipLaunchKernelGGL((k_wall<R, MK, EP2, false>), dim3(nb), dim3(64), 0, st, a, cs, cc);
    return hipSuccess;
}

template <typename R, int MK>
hipError_t launch_step_k(const StepArgs<R> &a, const CaseStatic *cs, CaseClock *cc, const Schedule &sch,
                         const TileArgs *ta, hipStream_t st, hipEvent_t *ev)
{
    // node ranges are multiples of CASE_ALIGN = 7 * 256, so every grid divides them evenly
    hipError_t e = hipSuccess;
    if (ev && (e = hipEventRecord(ev[0], st)) != hipSuccess) return e;
    if ((e = launch_stream_k<R, MK>(a, cs, cc, sch, ta, st)) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[1], st)) != hipSuccess) return e;
    if ((e = launch_wall_k<R, MK>(a, cs, cc, sch, st)) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[2], st)) != hipSuccess) return e;
    if ((e = launch_nodes_k<R, MK>(a, cs, cc, sch, st, ev ? ev[3] : nullptr)) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[4], st)) != hipSuccess) return e;
    return hipGetLastError();
}

template <typename R>
hipError_t launch_step(const StepArgs<R> &a, const CaseStatic *cs, CaseClock *cc, int motion_kind,
                       const Schedule &sch, const TileArgs *ta, hipStream_t st, hipEvent_t *ev)
{
    hipError_t e;
    switch (motion_kind) {
    case 1: e = launch_step_k<R, 1>(a, cs, cc, sch, ta, st, ev); break;
    case 2: e = launch_step_k<R, 2>(a, cs, cc, sch, ta, st, ev); break;
    case 3: e = launch_step_k<R, 3>(a, cs, cc, sch, ta, st, ev); break;
    default: e = launch_step_k<R, 0>(a, cs, cc, sch, ta, st, ev); break;
    }
    return e;
}

template <typename R>
hipError_t launch_stream_only(const StepArgs<R> &a, const CaseStatic *cs, const CaseClock *cc, int motion_kind,
                              const Schedule &sch, const TileArgs *ta, hipStream_t st)
{
    hipError_t e;
    switch (motion_kind) {
    case 1: e = launch_stream_k<R, 1>(a, cs, cc, sch, ta, st); break;
    case 2: e = launch_stream_k<R, 2>(a, cs, cc, sch, ta, st); break;
    case 3: e = launch_stream_k<R, 3>(a, cs, cc, sch, ta, st); break;
    default: e = launch_stream_k<R, 0>(a, cs, cc, sch, ta, st); break;
    }
    // the list the timed launches appended to is discarded
    if (e == hipSuccess) e = hipMemsetAsync(a.s.wcount, 0, sizeof(int), st);
    return e != hipSuccess ? e : hipGetLastError();
}

template <typename R>
hipError_t launch_node_kernels_only(const StepArgs<R> &a, const CaseStatic *cs, const CaseClock *cc,
                                    int motion_kind, const Schedule &sch, hipStream_t st)
{
    hipError_t e;
    switch (motion_kind) {
    case 1: e = launch_nodes_k<R, 1>(a, cs, cc, sch, st, nullptr); break;
    case 2: e = launch_nodes_k<R, 2>(a, cs, cc, sch, st, nullptr); break;
    case 3: e = launch_nodes_k<R, 3>(a, cs, cc, sch, st, nullptr); break;
    default: e = launch_nodes_k<R, 0>(a, cs, cc, sch, st, nullptr); break;
    }
    return e != hipSuccess ? e : hipGetLastError();
}

hipError_t launch_clock(const CaseStatic *cs, CaseClock *cc, int ncases, hipStream_t st)
{
    hipLaunchKernelGGL(k_clock, dim3((ncases + 63) / 64), dim3(64), 0, st, cs, cc, 0, ncases);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_stream_phase(const StepArgs<R> &a, const CaseStatic *cs, CaseClock *cc, int motion_kind,
                               const Schedule &sch, const TileArgs *ta, hipStream_t st)
{
    hipError_t e;
    switch (motion_kind) {
    case 1: e = launch_stream_k<R, 1>(a, cs, cc, sch, ta, st); break;
    case 2: e = launch_stream_k<R, 2>(a, cs, cc, sch, ta, st); break;
    case 3: e = launch_stream_k<R, 3>(a, cs, cc, sch, ta, st); break;
    default: e = launch_stream_k<R, 0>(a, cs, cc, sch, ta, st); break;
    }
    return e != hipSuccess ? e : hipGetLastError();
}

template <typename R>
hipError_t launch_wall_phase(const StepArgs<R> &a, const CaseStatic *cs, const CaseClock *cc, int motion_kind,
                             const Schedule &sch, hipStream_t st)
{
    hipError_t e;
    switch (motion_kind) {
    case 1: e = launch_wall_k<R, 1>(a, cs, cc, sch, st); break;
    case 2: e = launch_wall_k<R, 2>(a, cs, cc, sch, st); break;
    case 3: e = launch_wall_k<R, 3>(a, cs, cc, sch, st); break;
    default: e = launch_wall_k<R, 0>(a, cs, cc, sch, st); break;
    }
    return e != hipSuccess ? e : hipGetLastError();
}

template <typename R>
hipError_t launch_grad_phase(const StepArgs<R> &a, const CaseStatic *cs, const CaseClock *cc, int motion_kind,
                             const Schedule &sch, hipStream_t st)
{
    return launch_node_kernels_only<R>(a, cs, cc, motion_kind, sch, st);
}

hipError_t launch_freestream(CaseStatic *cs, int ncases, hipStream_t st)
{
    hipLaunchKernelGGL(k_freestream, dim3(ncases), dim3(64), 0, st, cs, ncases);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_init(const DevMesh &m, DevState<R> s, const CaseStatic *cs, const double *rho, const double *ux,
                       const double *uy, const double *T, int cur, hipStream_t st)
{
    hipLaunchKernelGGL(k_init<R>, dim3(blocks_for(m.N)), dim3(BLOCK), 0, st, m, s, cs, rho, ux, uy, T, cur);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_fold_x(const DevMesh &m, R *pop, R *X, const CaseStatic *cs, hipStream_t st)
{
    hipLaunchKernelGGL(k_fold_x<R>, dim3(blocks_for(m.N)), dim3(BLOCK), 0, st, m, pop, X, cs);
    return hipGetLastError();
}

hipError_t launch_move_mesh(const DevMesh &m, const CaseStatic *cs, const double *t_case, double *x, double *Jinv,
                            double *det, double *vg, int *err, hipStream_t st)
{
    hipLaunchKernelGGL(k_move_mesh, dim3(blocks_for(m.N)), dim3(BLOCK), 0, st, m, cs, t_case, x, Jinv, det, vg, err);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_forces(const DevMesh &m, const R *mac, const CaseStatic *cs, const CaseClock *cc, double *partial,
                         int nblocks, const int2 *case_blocks, double *out, hipStream_t st)
{
    if (nblocks > 0 && m.kind == ELEM_Q2)
        hipLaunchKernelGGL((k_forces<R, EQ2>), dim3(nblocks), dim3(BLOCK), 0, st, m, mac, cs, cc, partial);
    else if (nblocks > 0)
        hipLaunchKernelGGL((k_forces<R, EP2>), dim3(nblocks), dim3(BLOCK), 0, st, m, mac, cs, cc, partial);
    hipLaunchKernelGGL(k_sum_partials, dim3(m.ncases), dim3(64), 0, st, partial, case_blocks, m.ncases, out);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_convert(const R *src, double *dst, size_t n, int C, hipStream_t st, const DevMesh *m,
                          const CaseStatic *cs, const R *X)
{
    if (n == 0) return hipSuccess;
    if (bool(m) != bool(cs) || (m && C != NPOP) || (X && !m)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_convert<R>, dim3(blocks_for(n * C)), dim3(BLOCK), 0, st, src, dst, n, C, X,
                       m ? m->ncase : nullptr, cs);
    return hipGetLastError();
}
template <typename R>
hipError_t launch_convert_back(const double *src, R *dst, size_t n, int C, hipStream_t st, const DevMesh *m,
                               const CaseStatic *cs)
{
    if (n == 0) return hipSuccess;
    if (bool(m) != bool(cs) || (m && C != NPOP)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_convert_back<R>, dim3(blocks_for(n * C)), dim3(BLOCK), 0, st, src, dst, n, C,
                       m ? m->ncase : nullptr, cs);
    return hipGetLastError();
}

#define ALELB_INSTANTIATE(R)                                                                                          \
    template hipError_t launch_step<R>(const StepArgs<R> &, const CaseStatic *, CaseClock *, int, const Schedule &, \
                                       const TileArgs *, hipStream_t, hipEvent_t *);                                 \
    template hipError_t launch_stream_only<R>(const StepArgs<R> &, const CaseStatic *, const CaseClock *, int,      \
                                              const Schedule &, const TileArgs *, hipStream_t);                      \
    template hipError_t launch_node_kernels_only<R>(const StepArgs<R> &, const CaseStatic *, const CaseClock *, int, \
                                                    const Schedule &, hipStream_t);                                  \
    template hipError_t launch_stream_phase<R>(const StepArgs<R> &, const CaseStatic *, CaseClock *, int,           \
                                               const Schedule &, const TileArgs *, hipStream_t);                     \
    template hipError_t launch_wall_phase<R>(const StepArgs<R> &, const CaseStatic *, const CaseClock *, int,       \
                                             const Schedule &, hipStream_t);                                         \
    template hipError_t launch_grad_phase<R>(const StepArgs<R> &, const CaseStatic *, const CaseClock *, int,       \
                                             const Schedule &, hipStream_t);                                         \
    template hipError_t launch_init<R>(const DevMesh &, DevState<R>, const CaseStatic *, const double *,             \
                                       const double *, const double *, const double *, int, hipStream_t);            \
    template hipError_t launch_fold_x<R>(const DevMesh &, R *, R *, const CaseStatic *, hipStream_t);               \
    template hipError_t launch_forces<R>(const DevMesh &, const R *, const CaseStatic *, const CaseClock *,         \
                                         double *, int, const int2 *, double *, hipStream_t);                        \
    template hipError_t launch_convert<R>(const R *, double *, size_t, int, hipStream_t, const DevMesh *,           \
                                          const CaseStatic *, const R *);                                            \
    template hipError_t launch_convert_back<R>(const double *, R *, size_t, int, hipStream_t, const DevMesh *,      \
                                               const CaseStatic *);

ALELB_INSTANTIATE(float)
ALELB_INSTANTIATE(double)

}  // namespace alelb
