// gfx950 kernels of the ALE lattice-Boltzmann time step (Saadat & Karlin,
// arXiv 2002.04353).  One step is three launches over the nodes, all
// bandwidth-bound gathers on an unstructured P2 mesh:
//
//   k_stream   metrics at t^{n+1/2} and the transformed velocities
//              c^_i = J^-1 (c_i - v_g) (Sec. II, eq. Trasformed_Discrete_Vel),
//              departure points traced by the midpoint rule, element walk
//              (Sec. III, eq. NonLinear_Eq), P2 gather-interpolation
//              (eq. Propagation), Grad missing populations (Sec. IV.A,
//              tab. Neq_Moments) and the moments (eq. Temp).
//   k_grad1    W_a = (mu / rho T) d_a Q'_aaa through the owner element
//              (eqs. Xa, DeviationTerms, Ph_Derivative, FE_Derivative).
//   k_collide  X_a = -d_a W_a, then the two-population collision with
//              phi_i = A_ia X_a (eqs. feqn, geqn, feq, geq_gstar, Wi, Ai,
//              tab. Eq_Moments).
//
// R is the type of the populations and of the bulk arithmetic (float or
// double); coordinates, Jacobians, barycentrics and the force integral are
// always double.  Nodes are Morton-ordered, populations are stored as
// structure-of-arrays [18][N], one thread owns one node.
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

// ---- motion law (Sec. II): Jacobian J = dx/dX and grid velocity at (X, Y) ----
__device__ __forceinline__ void metric(const Motion &mo, const MotionTime &tf, double X, double Y,
                                       double J[4], double v[2])
{
    J[0] = 1.0; J[1] = 0.0; J[2] = 0.0; J[3] = 1.0;
    v[0] = 0.0; v[1] = 0.0;
    if (mo.kind == 1) {
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
    } else if (mo.kind == 2) {
        v[1] = tf.vy;
    } else if (mo.kind == 3) {
        const double Xc = mo.p[2], Yc = mo.p[3], r0 = mo.p[7], r1 = mo.p[8];
        const double c = tf.c, s = tf.s;
        const double rx = X - Xc, ry = Y - Yc;
        const double Dx = c * rx - s * ry + Xc - X;
        const double Dy = s * rx + c * ry + Yc - Y + tf.yoff;
        const double Vx = tf.thd * (-s * rx - c * ry);
        const double Vy = tf.thd * (c * rx - s * ry) + tf.vy;
        double b = 1.0, bX = 0.0, bY = 0.0;
        if (r1 > 0.0) {
            const double r = sqrt(rx * rx + ry * ry);
            const double sb = (r - r0) / (r1 - r0);
            if (sb >= 1.0) {
                b = 0.0;
            } else if (sb > 0.0) {
                b = 1.0 - sb * sb * sb * (10.0 - 15.0 * sb + 6.0 * sb * sb);
                const double db = -30.0 * sb * sb * (1.0 - sb) * (1.0 - sb);
                bX = db * rx / (r * (r1 - r0));
                bY = db * ry / (r * (r1 - r0));
            }
        }
        J[0] = 1.0 + b * (c - 1.0) + Dx * bX;
        J[1] = b * (-s) + Dx * bY;
        J[2] = b * s + Dy * bX;
        J[3] = 1.0 + b * (c - 1.0) + Dy * bY;
        v[0] = b * Vx; v[1] = b * Vy;
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
    const double det = J[0] * J[3] - J[1] * J[2];
    gx = (J[3] * gX - J[2] * gY) / det;
    gy = (-J[1] * gX + J[0] * gY) / det;
}

// ---- element walk over neighbours; P is updated across periodic edges ----
// returns the element (>= 0) with barycentrics l, or -1 wall, -2 far field, -4 cap
__device__ __forceinline__ int walk(const DevMesh &m, int e, double &Px, double &Py, double l[3])
{
    for (int it = 0; it < WALK_CAP; ++it) {
        const double2 v0 = m.eg[3 * e];
        const double2 a01 = m.eg[3 * e + 1];
        const double2 a23 = m.eg[3 * e + 2];
        const double dx = Px - v0.x, dy = Py - v0.y;
        l[1] = a01.x * dx + a01.y * dy;
        l[2] = a23.x * dx + a23.y * dy;
        l[0] = 1.0 - l[1] - l[2];
        int k = 0;
        double mn = l[0];
        if (l[1] < mn) { k = 1; mn = l[1]; }
        if (l[2] < mn) { k = 2; mn = l[2]; }
        if (mn >= -TAU_LOC) return e;
        const int4 t = m.et[e];
        const int n = k == 0 ? t.x : (k == 1 ? t.y : t.z);
        if (n < 0) return n;
        const int code = int((unsigned(t.w) >> (4 * k)) & 15u) - 4;
        if (code != 0) {
            const int c = code + 4;
            Px += double(c % 3 - 1) * m.Lx;
            Py += double(c / 3 - 1) * m.Ly;
        }
        e = n;
    }
    return -4;
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
template <typename R>
__device__ __forceinline__ R gform_i(int cx, int cy, R T, R M0, R Mx, R My, R Mxx, R Mxy, R Myy, R psi)
{
    const R fx = R(cx), fy = R(cy);
    const R W = wc(cx, T) * wc(cy, T);
    const R quad = ((Mxx - M0 * T) * (fx * fx - T) + R(2) * Mxy * fx * fy + (Myy - M0 * T) * (fy * fy - T)) /
                   (R(2) * T * T);
    return W * (M0 + (Mx * fx + My * fy) / T + quad) + psi;
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
    R M0, qx, qy, Rxx, Rxy, Ryy, Zx, Zy;
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
    p.Zx = rho * (R(1) - R(3) * T) * (T * T + R(2) * ux * ux * T + E * ux * ux) / T;
    p.Zy = rho * (R(1) - R(3) * T) * (T * T + R(2) * uy * uy * T + E * uy * uy) / T;
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
    // consecutive Morton tiles on the same XCD (workgroups are dealt round-robin over 8 XCDs)
    const int b = blockIdx.x;
    const int per = nblocks >> 3;
    return (b & 7) * per + (b >> 3);
}

// ---------------------------------------------------------------------------
// k_stream
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(BLOCK) void k_stream(StepArgs<R> a)
{
    const DevMesh &m = a.m;
    const int idx = xcd_block(gridDim.x) * BLOCK + threadIdx.x;
    if (idx >= m.N) return;
    const int N = m.N;
    const R *__restrict__ fin = a.s.pop[a.cur];
    const R *__restrict__ mprev = a.s.mac[a.cur];
    R *__restrict__ ft = a.s.ft;
    const double dt = a.ph.dt;

    const double2 Xa = m.X[idx];
    const int e0 = m.own[idx];
    const int info = m.oinfo[idx];
    const int scode = (info >> 3) & 15;
    const double P0x = Xa.x + double(scode % 3 - 1) * m.Lx;
    const double P0y = Xa.y + double(scode / 3 - 1) * m.Ly;

    double J[4], v[2];
    metric(a.mo, a.th, Xa.x, Xa.y, J, v);
    const double det = J[0] * J[3] - J[1] * J[2];
    if (!(det > 0.0)) atomicOr(a.s.err, ERR_JAC);
    const double Ji0 = J[3] / det, Ji1 = -J[1] / det, Ji2 = -J[2] / det, Ji3 = J[0] / det;

    R rho = 0, jx = 0, jy = 0, sg = 0;
    int mw = 0, mf = 0;
    bool have_tgt = false;
    // Grad targets and non-equilibrium moments (only built when a wall direction is missing)
    R t_rho = 0, t_ux = 0, t_uy = 0, t_T = 0, t_E = 0;
    R P1xx = 0, P1xy = 0, P1yy = 0, q1x = 0, q1y = 0, R1xx = 0, R1xy = 0, R1yy = 0;

    for (int i = 0; i < Q; ++i) {
        const int cx = cx_of(i), cy = cy_of(i);
        // transformed velocity at the arrival node, then at the trajectory midpoint
        double wx = double(cx) - v[0], wy = double(cy) - v[1];
        double chx = Ji0 * wx + Ji1 * wy, chy = Ji2 * wx + Ji3 * wy;
        const double Xm = Xa.x - 0.5 * dt * chx, Ym = Xa.y - 0.5 * dt * chy;
        double Jm[4], vm[2];
        metric(a.mo, a.th, Xm, Ym, Jm, vm);
        const double dm = Jm[0] * Jm[3] - Jm[1] * Jm[2];
        if (!(dm > 0.0)) atomicOr(a.s.err, ERR_JAC);
        wx = double(cx) - vm[0];
        wy = double(cy) - vm[1];
        chx = (Jm[3] / dm) * wx + (-Jm[1] / dm) * wy;
        chy = (-Jm[2] / dm) * wx + (Jm[0] / dm) * wy;
        double Px = P0x - dt * chx, Py = P0y - dt * chy;
        double l[3];
        const int e = walk(m, e0, Px, Py, l);
        R fv, gv;
        if (e >= 0) {
            double Nd[6];
            p2_shape(l, Nd);
            const int2 n01 = *reinterpret_cast<const int2 *>(m.en + 6 * e);
            const int2 n23 = *reinterpret_cast<const int2 *>(m.en + 6 * e + 2);
            const int2 n45 = *reinterpret_cast<const int2 *>(m.en + 6 * e + 4);
            const int nd[6] = {n01.x, n01.y, n23.x, n23.y, n45.x, n45.y};
            const R *fi = fin + size_t(i) * N;
            const R *gi = fin + size_t(Q + i) * N;
            fv = 0;
            gv = 0;
#pragma unroll
            for (int s = 0; s < 6; ++s) {
                fv += R(Nd[s]) * fi[nd[s]];
                gv += R(Nd[s]) * gi[nd[s]];
            }
        } else if (e == -2) {
            // far field: free-stream equilibrium (no non-equilibrium part)
            mf |= 1 << i;
            const R ri = R(a.ph.rho_inf), ux = R(a.ph.ux_inf), uy = R(a.ph.uy_inf), Ti = R(a.ph.T_inf);
            const R Ei = R(a.ph.Cv) * Ti + R(0.5) * (ux * ux + uy * uy);
            const GeqParts<R> gp = geq_parts(ri, ux, uy, Ti, Ei);
            fv = feq_i(cx, cy, ri, ux, uy, Ti);
            gv = gform_i(cx, cy, Ti, gp.M0, gp.qx, gp.qy, gp.Rxx, gp.Rxy, gp.Ryy, psi_i(cx, cy, gp));
        } else {
            if (e == -4) atomicOr(a.s.err, ERR_LOCATE);
            mw |= 1 << i;
            if (!have_tgt) {
                have_tgt = true;
                // targets: wall node -> wall velocity at t^{n+1}, rho and T at B;
                // any other node -> its own values of the previous step (Sec. IV.A)
                double J1[4], v1[2];
                metric(a.mo, a.t1, Xa.x, Xa.y, J1, v1);
                const int w = m.wid[idx];
                if (w >= 0) {
                    const int eb = m.bel[w];
                    double lb[3] = {m.blam[3 * w], m.blam[3 * w + 1], m.blam[3 * w + 2]};
                    double Nb[6];
                    p2_shape(lb, Nb);
                    double rb = 0.0, Tb = 0.0;
                    for (int s = 0; s < 6; ++s) {
                        const int nb = m.en[6 * eb + s];
                        rb += Nb[s] * double(mprev[nb]);
                        Tb += Nb[s] * double(mprev[3 * size_t(N) + nb]);
                    }
                    t_rho = R(rb);
                    t_T = R(Tb);
                    t_ux = R(v1[0]);
                    t_uy = R(v1[1]);
                } else {
                    t_rho = mprev[idx];
                    t_ux = mprev[size_t(N) + idx];
                    t_uy = mprev[2 * size_t(N) + idx];
                    t_T = mprev[3 * size_t(N) + idx];
                }
                // gradients of the previous-step u and T at the node, through the owner element
                const double2 a01 = m.eg[3 * e0 + 1], a23 = m.eg[3 * e0 + 2];
                double gN[6][2];
                p2_grad_at_node(info & 7, a01, a23, gN);
                double g[3][2] = {{0, 0}, {0, 0}, {0, 0}};
                for (int s = 0; s < 6; ++s) {
                    const int nb = m.en[6 * e0 + s];
                    const double u0 = double(mprev[size_t(N) + nb]);
                    const double u1 = double(mprev[2 * size_t(N) + nb]);
                    const double tt = double(mprev[3 * size_t(N) + nb]);
                    g[0][0] += u0 * gN[s][0]; g[0][1] += u0 * gN[s][1];
                    g[1][0] += u1 * gN[s][0]; g[1][1] += u1 * gN[s][1];
                    g[2][0] += tt * gN[s][0]; g[2][1] += tt * gN[s][1];
                }
                double dux_x, dux_y, duy_x, duy_y, dT_x, dT_y;
                to_physical(J1, g[0][0], g[0][1], dux_x, dux_y);
                to_physical(J1, g[1][0], g[1][1], duy_x, duy_y);
                to_physical(J1, g[2][0], g[2][1], dT_x, dT_y);
                // non-equilibrium moments of tab. Neq_Moments
                const R Cv = R(a.ph.Cv), Cp = R(a.ph.Cp);
                t_E = Cv * t_T + R(0.5) * (t_ux * t_ux + t_uy * t_uy);
                const R om = R(1) / (R(a.ph.mu) / (t_rho * t_T * R(dt)) + R(0.5));
                const R om1 = R(1) / (R(a.ph.mu) / (R(a.ph.Pr) * t_rho * t_T * R(dt)) + R(0.5));
                const R dxux = R(dux_x), dyux = R(dux_y), dxuy = R(duy_x), dyuy = R(duy_y);
                const R Sxx = R(2) * dxux, Syy = R(2) * dyuy, Sxy = dxuy + dyux;
                const R divu = dxux + dyuy;
                const R dEx = Cv * R(dT_x) + t_ux * dxux + t_uy * dxuy;
                const R dEy = Cv * R(dT_y) + t_ux * dyux + t_uy * dyuy;
                const R pre = -(R(1) / om) * t_rho * t_T;
                P1xx = pre * (Sxx - divu / Cv);
                P1xy = pre * Sxy;
                P1yy = pre * (Syy - divu / Cv);
                const R pr1 = -(R(2) / om1) * t_rho * t_T;
                R1xx = pr1 * (Sxx * (t_E + R(2) * t_T) + t_ux * dEx + t_ux * dEx);
                R1xy = pr1 * (Sxy * (t_E + R(2) * t_T) + t_ux * dEy + t_uy * dEx);
                R1yy = pr1 * (Syy * (t_E + R(2) * t_T) + t_uy * dEy + t_uy * dEy);
                q1x = -(R(2) / om1) * t_rho * Cp * t_T * R(dT_x) + R(2) * (t_ux * P1xx + t_uy * P1xy);
                q1y = -(R(2) / om1) * t_rho * Cp * t_T * R(dT_y) + R(2) * (t_ux * P1xy + t_uy * P1yy);
            }
            const GeqParts<R> gp = geq_parts(t_rho, t_ux, t_uy, t_T, t_E);
            const R f1 = gform_i(cx, cy, t_T, R(0), R(0), R(0), P1xx, P1xy, P1yy, R(0));
            const R g1 = gform_i(cx, cy, t_T, R(0), q1x, q1y, R1xx, R1xy, R1yy, R(0));
            fv = feq_i(cx, cy, t_rho, t_ux, t_uy, t_T) + R(dt) * f1;
            gv = gform_i(cx, cy, t_T, gp.M0, gp.qx, gp.qy, gp.Rxx, gp.Rxy, gp.Ryy, psi_i(cx, cy, gp)) +
                 R(dt) * g1;
        }
        ft[size_t(i) * N + idx] = fv;
        ft[size_t(Q + i) * N + idx] = gv;
        rho += fv;
        jx += R(cx) * fv;
        jy += R(cy) * fv;
        sg += gv;
    }
    // moments (eq. Temp): rho, u = j / rho, E = sum g / (2 rho), T = (E - u^2/2) / Cv
    R *__restrict__ mnew = a.s.mac[1 - a.cur];
    const R ux = jx / rho, uy = jy / rho;
    const R E = sg / (R(2) * rho);
    mnew[idx] = rho;
    mnew[size_t(N) + idx] = ux;
    mnew[2 * size_t(N) + idx] = uy;
    mnew[3 * size_t(N) + idx] = (E - R(0.5) * (ux * ux + uy * uy)) / R(a.ph.Cv);
    if (a.s.mask) a.s.mask[idx] = mw | (mf << 16);
}

// ---------------------------------------------------------------------------
// k_grad1: W_a = (mu / rho T) [g^-1 grad_X Q'_a]_a,  Q'_a = rho u_a (1 - 3T) - rho u_a^3
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(BLOCK) void k_grad1(StepArgs<R> a)
{
    const DevMesh &m = a.m;
    const int idx = xcd_block(gridDim.x) * BLOCK + threadIdx.x;
    if (idx >= m.N) return;
    const size_t N = m.N;
    const R *__restrict__ mac = a.s.mac[1 - a.cur];
    const int e = m.own[idx];
    const int slot = m.oinfo[idx] & 7;
    const double2 a01 = m.eg[3 * e + 1], a23 = m.eg[3 * e + 2];
    double gN[6][2];
    p2_grad_at_node(slot, a01, a23, gN);
    double gx0 = 0, gy0 = 0, gx1 = 0, gy1 = 0;
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        const int nb = m.en[6 * e + s];
        const R rho = mac[nb], ux = mac[N + nb], uy = mac[2 * N + nb], T = mac[3 * N + nb];
        const R qx = rho * ux * (R(1) - R(3) * T) - rho * ux * ux * ux;
        const R qy = rho * uy * (R(1) - R(3) * T) - rho * uy * uy * uy;
        gx0 += double(qx) * gN[s][0];
        gy0 += double(qx) * gN[s][1];
        gx1 += double(qy) * gN[s][0];
        gy1 += double(qy) * gN[s][1];
    }
    const double2 Xa = m.X[idx];
    double J[4], v[2];
    metric(a.mo, a.t1, Xa.x, Xa.y, J, v);
    double px, py, qx_, qy_;
    to_physical(J, gx0, gy0, px, py);
    to_physical(J, gx1, gy1, qx_, qy_);
    const R rho = mac[idx], T = mac[3 * N + idx];
    const R c = R(a.ph.mu) / (rho * T);
    a.s.W[idx] = c * R(px);
    a.s.W[N + idx] = c * R(qy_);
}

// ---------------------------------------------------------------------------
// k_collide: X_a = -[g^-1 grad_X W_a]_a, then eqs. feqn / geqn
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(BLOCK) void k_collide(StepArgs<R> a)
{
    const DevMesh &m = a.m;
    const int idx = xcd_block(gridDim.x) * BLOCK + threadIdx.x;
    if (idx >= m.N) return;
    const size_t N = m.N;
    const R *__restrict__ ft = a.s.ft;
    R *__restrict__ fout = a.s.pop[1 - a.cur];
    const bool collide = !(a.ph.flags & 1);

    R f[Q], g[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        f[i] = ft[size_t(i) * N + idx];
        g[i] = ft[size_t(Q + i) * N + idx];
    }
    if (!collide) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            fout[size_t(i) * N + idx] = f[i];
            fout[size_t(Q + i) * N + idx] = g[i];
        }
        return;
    }
    // correction field X through the owner element
    const int e = m.own[idx];
    const int slot = m.oinfo[idx] & 7;
    const double2 a01 = m.eg[3 * e + 1], a23 = m.eg[3 * e + 2];
    double gN[6][2];
    p2_grad_at_node(slot, a01, a23, gN);
    double wxx = 0, wxy = 0, wyx = 0, wyy = 0;
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        const int nb = m.en[6 * e + s];
        const double w0 = double(a.s.W[nb]), w1 = double(a.s.W[N + nb]);
        wxx += w0 * gN[s][0];
        wxy += w0 * gN[s][1];
        wyx += w1 * gN[s][0];
        wyy += w1 * gN[s][1];
    }
    const double2 Xa = m.X[idx];
    double J[4], v[2];
    metric(a.mo, a.t1, Xa.x, Xa.y, J, v);
    double d0x, d0y, d1x, d1y;
    to_physical(J, wxx, wxy, d0x, d0y);
    to_physical(J, wyx, wyy, d1x, d1y);
    const R Xx = R(-d0x), Xy = R(-d1y);
    a.s.Xc[idx] = Xx;
    a.s.Xc[N + idx] = Xy;

    // moments of the streamed populations
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
    const R ux = jx / rho, uy = jy / rho;
    const R E = sg / (R(2) * rho);
    const R T = (E - R(0.5) * (ux * ux + uy * uy)) / R(a.ph.Cv);
    const R dt = R(a.ph.dt);
    const R om = R(1) / (R(a.ph.mu) / (rho * T * dt) + R(0.5));
    const R om1 = R(1) / (R(a.ph.mu) / (R(a.ph.Pr) * rho * T * dt) + R(0.5));
    const GeqParts<R> gp = geq_parts(rho, ux, uy, T, E);
    // q* = q^eq + 2 u_b (P_ab - P^eq_ab)
    const R dPxx = pxx - (rho * ux * ux + rho * T);
    const R dPxy = pxy - rho * ux * uy;
    const R dPyy = pyy - (rho * uy * uy + rho * T);
    const R qsx = gp.qx + R(2) * (ux * dPxx + uy * dPxy);
    const R qsy = gp.qy + R(2) * (ux * dPxy + uy * dPyy);
    bool bad = false;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int cx = CX_[i], cy = CY_[i];
        const int c2 = cx * cx + cy * cy;
        const R ps = psi_i(cx, cy, gp);
        const R fe = feq_i(cx, cy, rho, ux, uy, T);
        const R ge = gform_i(cx, cy, T, gp.M0, gp.qx, gp.qy, gp.Rxx, gp.Rxy, gp.Ryy, ps);
        const R gq = gform_i(cx, cy, T, gp.M0, qsx, qsy, gp.Rxx, gp.Rxy, gp.Ryy, ps);
        const R Ax = R(cx) - R(0.5) * R(cx) * R(c2);
        const R Ay = R(cy) - R(0.5) * R(cy) * R(c2);
        const R fo = f[i] + om * (fe - f[i]) + dt * (Ax * Xx + Ay * Xy);
        const R go = g[i] + om * (ge - g[i]) + (om1 - om) * (gq - g[i]);
        fout[size_t(i) * N + idx] = fo;
        fout[size_t(Q + i) * N + idx] = go;
        bad |= !isfinite(fo) || !isfinite(go);
    }
    if ((a.ph.flags & 2) && bad) atomicOr(a.s.err, ERR_NONFINITE);
}

// ---------------------------------------------------------------------------
// initial condition: f = f^eq, g = g^eq (FP64 fields in internal order)
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(BLOCK) void k_init(int N, DevState<R> s, Phys ph, const double *rho,
                                                const double *ux, const double *uy, const double *T,
                                                int cur)
{
    const int idx = blockIdx.x * BLOCK + threadIdx.x;
    if (idx >= N) return;
    const R r = R(rho[idx]), u = R(ux[idx]), w = R(uy[idx]), t = R(T[idx]);
    const R E = R(ph.Cv) * t + R(0.5) * (u * u + w * w);
    const GeqParts<R> gp = geq_parts(r, u, w, t, E);
    R *p = s.pop[cur];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int cx = CX_[i], cy = CY_[i];
        p[size_t(i) * N + idx] = feq_i(cx, cy, r, u, w, t);
        p[size_t(Q + i) * N + idx] = gform_i(cx, cy, t, gp.M0, gp.qx, gp.qy, gp.Rxx, gp.Rxy, gp.Ryy,
                                             psi_i(cx, cy, gp));
    }
    R *mc = s.mac[cur];
    mc[idx] = r;
    mc[size_t(N) + idx] = u;
    mc[2 * size_t(N) + idx] = w;
    mc[3 * size_t(N) + idx] = t;
}

__global__ __launch_bounds__(BLOCK) void k_move_mesh(DevMesh m, Motion mo, MotionTime tf, double *x,
                                                     double *Jinv, double *det, double *vg, int *err)
{
    const int idx = blockIdx.x * BLOCK + threadIdx.x;
    if (idx >= m.N) return;
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
// forces: traction on straight P2 wall edges, Simpson weights 1/6 4/6 1/6,
// p = rho T, tau = mu (S - (1/Cv) div u I), gradients from the edge's element;
// per-block sums in a fixed order, then one block sums the partials.
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(BLOCK) void k_forces(DevMesh m, const R *mac, Phys ph, Motion mo,
                                                  MotionTime tf, double *partial)
{
    __shared__ double red[6][BLOCK];
    const int w = blockIdx.x * BLOCK + threadIdx.x;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    if (w < m.NWE) {
        const size_t N = m.N;
        const int2 we = m.wedge[w];
        const int e = we.x, k = we.y;
        const int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
        const double2 a01 = m.eg[3 * e + 1], a23 = m.eg[3 * e + 2];
        const double4 ab = m.wxy[w];
        double xa, ya, xb, yb;
        position(mo, tf, ab.x, ab.y, xa, ya);
        position(mo, tf, ab.z, ab.w, xb, yb);
        const double dx = xb - xa, dy = yb - ya;
        const double len = sqrt(dx * dx + dy * dy);
        const double nx = -dy / len, ny = dx / len;
        const int slots[3] = {k1, 3 + k, k2};
        const double wts[3] = {1.0 / 6.0, 4.0 / 6.0, 1.0 / 6.0};
        for (int j = 0; j < 3; ++j) {
            const int s = slots[j];
            double gN[6][2];
            p2_grad_at_node(s, a01, a23, gN);
            const double X0 = j == 0 ? ab.x : (j == 2 ? ab.z : 0.5 * (ab.x + ab.z));
            const double Y0 = j == 0 ? ab.y : (j == 2 ? ab.w : 0.5 * (ab.y + ab.w));
            double gu[2][2] = {{0, 0}, {0, 0}};
            for (int q = 0; q < 6; ++q) {
                const int nb = m.en[6 * e + q];
                const double u0 = double(mac[N + nb]), u1 = double(mac[2 * N + nb]);
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
            for (int c = 0; c < 2; ++c)
                for (int d = 0; d < 2; ++d)
                    tau[c][d] = ph.mu * (G[c][d] + G[d][c] - (c == d ? divu / ph.Cv : 0.0));
            const int an = m.en[6 * e + s];
            const double pr = double(mac[an]) * double(mac[3 * N + an]);
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
    for (int c = 0; c < 6; ++c) red[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int half = BLOCK / 2; half > 0; half >>= 1) {
        if (threadIdx.x < half)
#pragma unroll
            for (int c = 0; c < 6; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + half];
        __syncthreads();
    }
    if (threadIdx.x < 6) partial[6 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void k_sum_partials(const double *partial, int nb, double *out)
{
    if (threadIdx.x < 6) {
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += partial[6 * b + threadIdx.x];
        out[threadIdx.x] = s;
    }
}

template <typename R>
__global__ void k_convert(const R *src, double *dst, size_t n)
{
    const size_t i = size_t(blockIdx.x) * BLOCK + threadIdx.x;
    if (i < n) dst[i] = double(src[i]);
}
template <typename R>
__global__ void k_convert_back(const double *src, R *dst, size_t n)
{
    const size_t i = size_t(blockIdx.x) * BLOCK + threadIdx.x;
    if (i < n) dst[i] = R(src[i]);
}

inline unsigned blocks_for(size_t n) { return unsigned((n + BLOCK - 1) / BLOCK); }
inline unsigned blocks_xcd(size_t n) { return (blocks_for(n) + 7u) & ~7u; }

}  // namespace

MotionTime motion_time(const Motion &mo, double t)
{
    MotionTime tf{0, 0, 0, 0, 0};
    if (mo.kind == 1) {
        tf.s = std::sin(2.0 * PI * t / mo.p[3]);
        tf.c = std::cos(2.0 * PI * t / mo.p[3]);
    } else if (mo.kind == 2) {
        tf.yoff = -mo.p[0] * std::sin(mo.p[1] * t + mo.p[2]);
        tf.vy = -mo.p[0] * mo.p[1] * std::cos(mo.p[1] * t + mo.p[2]);
    } else if (mo.kind == 3) {
        const double A = mo.p[0], w = mo.p[1], php = mo.p[4], h = mo.p[5], phh = mo.p[6];
        const double th = A * std::sin(w * t + php);
        tf.c = std::cos(th);
        tf.s = std::sin(th);
        tf.thd = A * w * std::cos(w * t + php);
        tf.yoff = -h * std::sin(w * t + phh);
        tf.vy = -h * w * std::cos(w * t + phh);
    }
    return tf;
}

template <typename R>
hipError_t launch_step(const StepArgs<R> &a, hipStream_t st, hipEvent_t *ev)
{
    const unsigned nb = blocks_xcd(a.m.N);
    hipError_t e = hipSuccess;
    if (ev && (e = hipEventRecord(ev[0], st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_stream<R>, dim3(nb), dim3(BLOCK), 0, st, a);
    if (ev && (e = hipEventRecord(ev[1], st)) != hipSuccess) return e;
    if (!(a.ph.flags & 1)) hipLaunchKernelGGL(k_grad1<R>, dim3(nb), dim3(BLOCK), 0, st, a);
    if (ev && (e = hipEventRecord(ev[2], st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_collide<R>, dim3(nb), dim3(BLOCK), 0, st, a);
    if (ev && (e = hipEventRecord(ev[3], st)) != hipSuccess) return e;
    return hipGetLastError();
}

template <typename R>
hipError_t launch_init(const DevMesh &m, DevState<R> s, const Phys &ph, const double *rho,
                       const double *ux, const double *uy, const double *T, int cur, hipStream_t st)
{
    hipLaunchKernelGGL(k_init<R>, dim3(blocks_for(m.N)), dim3(BLOCK), 0, st, m.N, s, ph, rho, ux, uy, T, cur);
    return hipGetLastError();
}

hipError_t launch_move_mesh(const DevMesh &m, const Motion &mo, MotionTime tf, double *x, double *Jinv,
                            double *det, double *vg, int *err, hipStream_t st)
{
    hipLaunchKernelGGL(k_move_mesh, dim3(blocks_for(m.N)), dim3(BLOCK), 0, st, m, mo, tf, x, Jinv, det, vg, err);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_forces(const DevMesh &m, const R *mac, const Phys &ph, const Motion &mo, MotionTime tf,
                         double *partial, int nblocks, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_forces<R>, dim3(nblocks), dim3(BLOCK), 0, st, m, mac, ph, mo, tf, partial);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, st, partial, nblocks, out);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_convert(const R *src, double *dst, size_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_convert<R>, dim3(blocks_for(n)), dim3(BLOCK), 0, st, src, dst, n);
    return hipGetLastError();
}
template <typename R>
hipError_t launch_convert_back(const double *src, R *dst, size_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_convert_back<R>, dim3(blocks_for(n)), dim3(BLOCK), 0, st, src, dst, n);
    return hipGetLastError();
}

template hipError_t launch_step<float>(const StepArgs<float> &, hipStream_t, hipEvent_t *);
template hipError_t launch_step<double>(const StepArgs<double> &, hipStream_t, hipEvent_t *);
template hipError_t launch_init<float>(const DevMesh &, DevState<float>, const Phys &, const double *,
                                       const double *, const double *, const double *, int, hipStream_t);
template hipError_t launch_init<double>(const DevMesh &, DevState<double>, const Phys &, const double *,
                                        const double *, const double *, const double *, int, hipStream_t);
template hipError_t launch_forces<float>(const DevMesh &, const float *, const Phys &, const Motion &,
                                         MotionTime, double *, int, double *, hipStream_t);
template hipError_t launch_forces<double>(const DevMesh &, const double *, const Phys &, const Motion &,
                                          MotionTime, double *, int, double *, hipStream_t);
template hipError_t launch_convert<float>(const float *, double *, size_t, hipStream_t);
template hipError_t launch_convert<double>(const double *, double *, size_t, hipStream_t);
template hipError_t launch_convert_back<float>(const double *, float *, size_t, hipStream_t);
template hipError_t launch_convert_back<double>(const double *, double *, size_t, hipStream_t);

}  // namespace alelb
