/*
 * Plain FP64 CPU oracle of one ALE lattice-Boltzmann time step.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the CPU
 * baseline leg of the benchmark, never by the product path.  It is written
 * from the paper (Saadat & Karlin, arXiv 2002.04353) step by step, in the
 * paper's order and notation, with no blocking or fusion, so that each pass
 * can be read against the section or equation it cites.  Build: plain C99,
 * -O2, -ffp-contract=off, OpenMP over nodes inside each pass.
 *
 * One step n -> n+1 (t^n = t0 + n dt):
 *   1. mapping metrics J = dx/dX, grid velocity v_g = dG/dt       (Sec. II)
 *   2. transformed velocities c^_i = J^-1 (c_i - v_g), departure point
 *      X - dt c^_i, traced by the midpoint rule at t^{n+1/2}  (Sec. II, eq. Trasformed_Discrete_Vel)
 *   3. locate the departure point's element (visibility walk)     (Sec. III, eq. NonLinear_Eq)
 *   4. second-order finite-element interpolation                  (Sec. III, eq. Propagation)
 *   5. missing populations by Grad's approximation                (Sec. IV.A, tab. Neq_Moments)
 *   6. moments rho, u, E, T                                       (Sec. IV, eq. Temp)
 *   7-8. correction term phi_i through two FE derivative passes   (Sec. IV, eqs. Xa, Ai, DeviationTerms,
 *                                                                  Ph_Derivative, FE_Derivative)
 *   9. two-population collision                                   (Sec. IV, eqs. feqn, geqn, feq, geq_gstar, Wi,
 *                                                                  tab. Eq_Moments)
 *  10. wall force integral (on request)                           (Sec. V.B / V.C coefficient definitions)
 */
#include "alelb_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 9
static const int CX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double PI = 3.14159265358979323846;
static const double TAU_LOC = 1e-12;  /* walk acceptance: min barycentric >= -TAU_LOC */
static const int WALK_CAP = 256;

struct orc {
    int nn, ne, nwe;
    int kind;           /* 0: 6-node P2 triangle, 1: 9-node Q2 quadrilateral */
    int nv, nf;         /* nodes and edges per element: 6, 3 or 9, 4 */
    double *X;          /* [nn][2] */
    int *elem;          /* [ne][nv] */
    int *nbr;           /* [ne][nf] */
    signed char *psh;   /* [ne][nf] */
    double period[2];
    int *wedge;         /* [nwe][2] */
    orc_params_t p;
    double Cv, Cp;
    /* derived geometry */
    double *ev;         /* P2: [ne][3][2] vertex coordinates in the element's frame */
    double *Ainv;       /* P2: [ne][4]: (l1, l2) = Ainv (P - v0) */
    double *qc;         /* Q2: [ne][4][2] corner coordinates in the element's frame */
    double *area;       /* [ne] */
    int *owner;         /* [nn] */
    int *oslot;         /* [nn] local index of the node in its owner element */
    double *opos;       /* [nn][2] node position in the owner's frame */
    int *wid;           /* [nn] wall-node index or -1 */
    int nw;
    double *wnorm;      /* [nw][2] computational into-fluid unit normal */
    int *bel;           /* [nw] element holding point B */
    double *blam;       /* [nw][3] local coordinates of B (barycentrics, or xi, eta) */
    /* state */
    double *f, *g;      /* [nn][9] post-collision populations */
    double *M;          /* [nn][4] rho ux uy T of the last completed step */
    double *ft, *gt;    /* [nn][9] streamed populations */
    double *Mn;         /* [nn][4] */
    double *W;          /* [nn][2] */
    double *Xa;         /* [nn][2] */
    int *mw, *mf;       /* [nn] missing-direction masks (wall / far field) */
    long step;
    double t;
    char err[256];
};

/* ------------------------------------------------------------------------ */
/* mapping x = G(X, t), its Jacobian J = dx/dX and grid velocity v = dG/dt   */
/* (Sec. II; motion laws of Sec. V.A, eq. Plunge_eq and Sec. V.C)            */
/* ------------------------------------------------------------------------ */
void orc_motion(const orc_params_t *p, double X, double Y, double t, double *x, double *J, double *v)
{
    const double *m = p->motion_p;
    x[0] = X; x[1] = Y;
    J[0] = 1.0; J[1] = 0.0; J[2] = 0.0; J[3] = 1.0;
    v[0] = 0.0; v[1] = 0.0;
    if (p->motion == ORC_MOTION_SINE) {
        /* x = X + a sin(2 pi X/Lx) sin(2 pi Y/Ly) sin(2 pi t/Tp), y = Y + (same) */
        double a = m[0], Lx = m[1], Ly = m[2], Tp = m[3];
        double sx = sin(2.0 * PI * X / Lx), cx = cos(2.0 * PI * X / Lx);
        double sy = sin(2.0 * PI * Y / Ly), cy = cos(2.0 * PI * Y / Ly);
        double st = sin(2.0 * PI * t / Tp), ct = cos(2.0 * PI * t / Tp);
        double d = a * sx * sy * st;
        double dX = a * (2.0 * PI / Lx) * cx * sy * st;
        double dY = a * (2.0 * PI / Ly) * sx * cy * st;
        double dt_ = a * sx * sy * (2.0 * PI / Tp) * ct;
        x[0] = X + d; x[1] = Y + d;
        J[0] = 1.0 + dX; J[1] = dY;
        J[2] = dX;       J[3] = 1.0 + dY;
        v[0] = dt_; v[1] = dt_;
    } else if (p->motion == ORC_MOTION_PLUNGE) {
        /* x = X, y = Y - h sin(w t + phase) */
        double h = m[0], w = m[1], ph = m[2];
        x[1] = Y - h * sin(w * t + ph);
        v[1] = -h * w * cos(w * t + ph);
    } else if (p->motion == ORC_MOTION_PITCH_PLUNGE) {
        /* rotation by theta = A sin(w t + phase_p) about (Xc, Yc), plus a plunge
           (0, -h sin(w t + phase_h)); blended to rest between radii r0 and r1
           (r1 <= 0: rigid everywhere) */
        double A = m[0], w = m[1], Xc = m[2], Yc = m[3], php = m[4], h = m[5], phh = m[6];
        double r0 = m[7], r1 = m[8];
        double th = A * sin(w * t + php), thd = A * w * cos(w * t + php);
        double c = cos(th), s = sin(th);
        double rx = X - Xc, ry = Y - Yc;
        double Dx = c * rx - s * ry + Xc - X;
        double Dy = s * rx + c * ry + Yc - Y - h * sin(w * t + phh);
        double Vx = thd * (-s * rx - c * ry);
        double Vy = thd * (c * rx - s * ry) - h * w * cos(w * t + phh);
        double b = 1.0, bX = 0.0, bY = 0.0;
        if (r1 > 0.0) {
            double r = sqrt(rx * rx + ry * ry);
            double sb = (r - r0) / (r1 - r0);
            if (sb <= 0.0) {
                b = 1.0;
            } else if (sb >= 1.0) {
                b = 0.0;
            } else {
                b = 1.0 - sb * sb * sb * (10.0 - 15.0 * sb + 6.0 * sb * sb);
                double db = -30.0 * sb * sb * (1.0 - sb) * (1.0 - sb);
                bX = db * rx / (r * (r1 - r0));
                bY = db * ry / (r * (r1 - r0));
            }
        }
        x[0] = X + b * Dx; x[1] = Y + b * Dy;
        J[0] = 1.0 + b * (c - 1.0) + Dx * bX;
        J[1] = b * (-s) + Dx * bY;
        J[2] = b * s + Dy * bX;
        J[3] = 1.0 + b * (c - 1.0) + Dy * bY;
        v[0] = b * Vx; v[1] = b * Vy;
    }
}

static int inv2(const double *J, double *Ji, double *det)
{
    double d = J[0] * J[3] - J[1] * J[2];
    *det = d;
    if (!(d > 0.0)) return -1;
    Ji[0] = J[3] / d;  Ji[1] = -J[1] / d;
    Ji[2] = -J[2] / d; Ji[3] = J[0] / d;
    return 0;
}

/* physical gradient from the computational one: grad_x K = g^-1 grad_X K with
   g^-1 = (1/det)[[y_Y, -y_X], [-x_Y, x_X]] (Sec. II, eq. g_inv; eq. Ph_Derivative) */
static int phys_grad(const orc_params_t *p, double X, double Y, double t, const double *gX, double *gx)
{
    double x[2], J[4], v[2];
    orc_motion(p, X, Y, t, x, J, v);
    double det = J[0] * J[3] - J[2] * J[1];
    if (!(det > 0.0)) return -1;
    gx[0] = (J[3] * gX[0] - J[2] * gX[1]) / det;
    gx[1] = (-J[1] * gX[0] + J[0] * gX[1]) / det;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* P2 triangle: shape functions and their gradients (Sec. III, eq. Propagation)
 * local nodes v0 v1 v2 m12 m20 m01; with barycentrics l_k:
 *   N_k = l_k (2 l_k - 1),  N_{3+k} = 4 l_{k+1} l_{k+2}                       */
/* ------------------------------------------------------------------------ */
void orc_p2_shape(const double *l, double *N)
{
    for (int k = 0; k < 3; ++k) {
        N[k] = l[k] * (2.0 * l[k] - 1.0);
        N[3 + k] = 4.0 * l[(k + 1) % 3] * l[(k + 2) % 3];
    }
}

static void p2_grad_shape(const double *l, const double *A, double gN[6][2])
{
    double gl[3][2];
    gl[1][0] = A[0]; gl[1][1] = A[1];
    gl[2][0] = A[2]; gl[2][1] = A[3];
    gl[0][0] = -A[0] - A[2]; gl[0][1] = -A[1] - A[3];
    for (int k = 0; k < 3; ++k) {
        int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
        for (int d = 0; d < 2; ++d) {
            gN[k][d] = (4.0 * l[k] - 1.0) * gl[k][d];
            gN[3 + k][d] = 4.0 * (l[k1] * gl[k2][d] + l[k2] * gl[k1][d]);
        }
    }
}

static void node_lambda(int slot, double *l)
{
    l[0] = l[1] = l[2] = 0.0;
    if (slot < 3) {
        l[slot] = 1.0;
    } else {
        l[(slot - 3 + 1) % 3] = 0.5;
        l[(slot - 3 + 2) % 3] = 0.5;
    }
}

/* ------------------------------------------------------------------------ */
/* Q2 quadrilateral (the element of Sec. III): 9-node Lagrange interpolation
 * on the reference square [-1,1]^2 with bilinear geometry from the corners.
 * Nodes: corners 0..3 at (-1,-1) (1,-1) (1,1) (-1,1), node 4+k at the middle
 * of edge k (corner k to corner k+1), node 8 at the centre.
 *   N_s(xi, eta) = L_{xi_s}(xi) L_{eta_s}(eta), L_{-1}(t) = t (t-1)/2,
 *   L_0(t) = (1-t)(1+t), L_1(t) = t (t+1)/2;
 *   x(xi, eta) = sum_k (1 + xi_k xi)(1 + eta_k eta)/4 c_k.                   */
/* ------------------------------------------------------------------------ */
static const double QXI[9] = {-1, 1, 1, -1, 0, 1, 0, -1, 0};
static const double QETA[9] = {-1, -1, 1, 1, -1, 0, 1, 0, 0};

static void lagrange3(double t, double *L, double *dL)
{
    L[0] = 0.5 * t * (t - 1.0);
    L[1] = (1.0 - t) * (1.0 + t);
    L[2] = 0.5 * t * (t + 1.0);
    dL[0] = t - 0.5;
    dL[1] = -2.0 * t;
    dL[2] = t + 0.5;
}

void orc_q2_shape(const double *xe, double *N)
{
    double Lx[3], dLx[3], Ly[3], dLy[3];
    lagrange3(xe[0], Lx, dLx);
    lagrange3(xe[1], Ly, dLy);
    for (int s = 0; s < 9; ++s) N[s] = Lx[(int)QXI[s] + 1] * Ly[(int)QETA[s] + 1];
}

/* bilinear map of the corners c[4][2]: position and J = [dx/dxi dx/deta; dy/dxi dy/deta] */
static void q2_map(const double *c, double xi, double eta, double *x, double *J)
{
    x[0] = x[1] = 0.0;
    J[0] = J[1] = J[2] = J[3] = 0.0;
    for (int k = 0; k < 4; ++k) {
        double b = 0.25 * (1.0 + QXI[k] * xi) * (1.0 + QETA[k] * eta);
        double bxi = 0.25 * QXI[k] * (1.0 + QETA[k] * eta);
        double beta = 0.25 * QETA[k] * (1.0 + QXI[k] * xi);
        for (int d = 0; d < 2; ++d) {
            x[d] += b * c[2 * k + d];
            J[2 * d] += bxi * c[2 * k + d];
            J[2 * d + 1] += beta * c[2 * k + d];
        }
    }
}

/* eq. NonLinear_Eq: x(xi, eta) = P by Newton's method from the centre */
static void q2_local(const double *c, const double *P, double *xe)
{
    double xi = 0.0, eta = 0.0;
    for (int it = 0; it < 8; ++it) {
        double x[2], J[4];
        q2_map(c, xi, eta, x, J);
        double r0 = x[0] - P[0], r1 = x[1] - P[1];
        double det = J[0] * J[3] - J[1] * J[2];
        double dxi = (J[3] * r0 - J[1] * r1) / det;
        double deta = (-J[2] * r0 + J[0] * r1) / det;
        xi -= dxi;
        eta -= deta;
        if (fabs(dxi) + fabs(deta) < 1e-14) break;
    }
    xe[0] = xi;
    xe[1] = eta;
    xe[2] = 0.0;
}

/* computational gradients of the 9 shape functions at local node `slot` */
static void q2_grad_slot(const double *c, int slot, double gN[9][2])
{
    double xe[2] = {QXI[slot], QETA[slot]};
    double Lx[3], dLx[3], Ly[3], dLy[3], x[2], J[4];
    lagrange3(xe[0], Lx, dLx);
    lagrange3(xe[1], Ly, dLy);
    q2_map(c, xe[0], xe[1], x, J);
    double det = J[0] * J[3] - J[1] * J[2];
    for (int s = 0; s < 9; ++s) {
        double dxi = dLx[(int)QXI[s] + 1] * Ly[(int)QETA[s] + 1];
        double deta = Lx[(int)QXI[s] + 1] * dLy[(int)QETA[s] + 1];
        /* [dN/dx, dN/dy] = J^-T [dN/dxi, dN/deta] */
        gN[s][0] = (J[3] * dxi - J[2] * deta) / det;
        gN[s][1] = (-J[1] * dxi + J[0] * deta) / det;
    }
}

/* ---- element-kind dispatch ---- */
static void elem_shape(const orc_t *o, const double *loc, double *N)
{
    if (o->kind == 0) orc_p2_shape(loc, N);
    else orc_q2_shape(loc, N);
}

static void elem_grad_slot(const orc_t *o, int e, int slot, double gN[9][2])
{
    if (o->kind == 0) {
        double l[3], g6[6][2];
        node_lambda(slot, l);
        p2_grad_shape(l, o->Ainv + 4 * e, g6);
        for (int s = 0; s < 6; ++s) { gN[s][0] = g6[s][0]; gN[s][1] = g6[s][1]; }
    } else {
        q2_grad_slot(o->qc + 8 * e, slot, gN);
    }
}

/* position of local node `slot` in the element's frame */
static void elem_node_pos(const orc_t *o, int e, int slot, double *pos)
{
    if (o->kind == 0) {
        const double *v = o->ev + 6 * e;
        if (slot < 3) {
            pos[0] = v[2 * slot]; pos[1] = v[2 * slot + 1];
        } else {
            int k1 = (slot - 3 + 1) % 3, k2 = (slot - 3 + 2) % 3;
            pos[0] = 0.5 * (v[2 * k1] + v[2 * k2]);
            pos[1] = 0.5 * (v[2 * k1 + 1] + v[2 * k2 + 1]);
        }
    } else {
        double J[4];
        q2_map(o->qc + 8 * e, QXI[slot], QETA[slot], pos, J);
    }
}

/* edge k: its three nodes (end, middle, end) and end points, counter-clockwise */
static void elem_edge(const orc_t *o, int e, int k, int *slots, double *a, double *b)
{
    if (o->kind == 0) {
        int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
        slots[0] = k1; slots[1] = 3 + k; slots[2] = k2;
    } else {
        slots[0] = k; slots[1] = 4 + k; slots[2] = (k + 1) % 4;
    }
    elem_node_pos(o, e, slots[0], a);
    elem_node_pos(o, e, slots[2], b);
}

/* ------------------------------------------------------------------------ */
/* locate: visibility walk over neighbours (Sec. III, eq. NonLinear_Eq: for a
 * straight-sided triangle the map is affine and the barycentrics are exact;
 * for the quadrilateral it is solved by Newton's method)                    */
/* ------------------------------------------------------------------------ */
static void barycentric(const orc_t *o, int e, const double *P, double *l)
{
    const double *v0 = o->ev + 6 * e;
    const double *A = o->Ainv + 4 * e;
    double dx = P[0] - v0[0], dy = P[1] - v0[1];
    l[1] = A[0] * dx + A[1] * dy;
    l[2] = A[2] * dx + A[3] * dy;
    l[0] = 1.0 - l[1] - l[2];
}

static void apply_shift(const orc_t *o, int code, double *P)
{
    if (code == 0) return;
    int c = code + 4;
    int sx = c % 3 - 1, sy = c / 3 - 1;
    P[0] += sx * o->period[0];
    P[1] += sy * o->period[1];
}

/* Which side of element e's edges P lies on.  Triangle: the barycentrics;
 * edge k is opposite vertex k.  Quadrilateral (straight edges: the geometry
 * is bilinear): s_k = cross(c_{k+1} - c_k, P - c_k) / (2 area), which is
 * >= 0 on the element's side of edge k (the same form as a barycentric).
 * Returns the smallest value, with its edge in *face (lowest on ties); P lies
 * in e when it is >= -TAU_LOC, and then loc holds P's local coordinates
 * (barycentrics, or (xi, eta) of eq. NonLinear_Eq by Newton's method). */
static double elem_side(const orc_t *o, int e, const double *P, double *loc, int *face)
{
    double v[4];
    int nf;
    if (o->kind == 0) {
        barycentric(o, e, P, loc);
        v[0] = loc[0]; v[1] = loc[1]; v[2] = loc[2];
        nf = 3;
    } else {
        const double *c = o->qc + 8 * e;
        for (int k = 0; k < 4; ++k) {
            const double *pa = c + 2 * k, *pb = c + 2 * ((k + 1) % 4);
            v[k] = ((pb[0] - pa[0]) * (P[1] - pa[1]) - (pb[1] - pa[1]) * (P[0] - pa[0])) / (2.0 * o->area[e]);
        }
        nf = 4;
    }
    int k = 0;
    for (int j = 1; j < nf; ++j)
        if (v[j] < v[k]) k = j;
    *face = k;
    if (o->kind == 1 && v[k] >= -TAU_LOC) q2_local(o->qc + 8 * e, P, loc);
    return v[k];
}

static int elem_test(const orc_t *o, int e, const double *P, double *loc, int *face)
{
    return elem_side(o, e, P, loc, face) >= -TAU_LOC;
}

int orc_locate(const orc_t *o, int32_t e, const double *Pin, int32_t *e_out, double *l, int32_t *steps)
{
    double P[2] = {Pin[0], Pin[1]};
    for (int it = 0; it < WALK_CAP; ++it) {
        int k;
        if (elem_test(o, e, P, l, &k)) {
            *e_out = e;
            if (steps) *steps = it;
            return 0;
        }
        int n = o->nbr[o->nf * e + k];
        if (n < 0) {
            *e_out = e;
            if (steps) *steps = it;
            return n; /* -1 wall, -2 far field */
        }
        apply_shift(o, o->psh[o->nf * e + k], P);
        e = n;
    }
    return ORC_ELOCATE;
}

int orc_brute_locate(const orc_t *o, const double *P, int32_t *e_out, double *l)
{
    int best = -1;
    double bestm = -1e300, bl[3] = {0, 0, 0};
    int nsx = o->period[0] > 0 ? 1 : 0, nsy = o->period[1] > 0 ? 1 : 0;
    for (int e = 0; e < o->ne; ++e) {
        for (int sx = -nsx; sx <= nsx; ++sx)
            for (int sy = -nsy; sy <= nsy; ++sy) {
                double Q2[2] = {P[0] + sx * o->period[0], P[1] + sy * o->period[1]};
                double lam[3] = {0, 0, 0};
                int face;
                double m = elem_side(o, e, Q2, lam, &face);
                if (m > bestm) {
                    bestm = m; best = e;
                    bl[0] = lam[0]; bl[1] = lam[1]; bl[2] = lam[2];
                }
            }
    }
    *e_out = best;
    l[0] = bl[0]; l[1] = bl[1]; l[2] = bl[2];
    return bestm >= -TAU_LOC ? 0 : -1;
}

/* ------------------------------------------------------------------------ */
/* equilibria (Sec. IV, eqs. feq, geq_gstar, Wi, tab. Eq_Moments)           */
/* ------------------------------------------------------------------------ */
static double Phi(int c, double u, double T)
{
    if (c == 0) return 1.0 - (u * u + T);
    return (c * u + u * u + T) / 2.0;
}

static double Wc(int c, double T) { return c == 0 ? 1.0 - T : T / 2.0; }

void orc_feq(double rho, double ux, double uy, double T, double *f)
{
    for (int i = 0; i < Q; ++i) f[i] = rho * Phi(CX[i], ux, T) * Phi(CY[i], uy, T);
}

/* general form G_i(M0, M_a, M_ab, Psi_i); Mab = {xx, xy, yy} */
static void Gform(double T, double M0, const double *Ma, const double *Mab, const double *Psi, double *out)
{
    for (int i = 0; i < Q; ++i) {
        double cx = CX[i], cy = CY[i];
        double W = Wc(CX[i], T) * Wc(CY[i], T);
        double quad = ((Mab[0] - M0 * T) * (cx * cx - T)
                       + 2.0 * Mab[1] * cx * cy
                       + (Mab[2] - M0 * T) * (cy * cy - T)) / (2.0 * T * T);
        out[i] = W * (M0 + (Ma[0] * cx + Ma[1] * cy) / T + quad) + (Psi ? Psi[i] : 0.0);
    }
}

/* B_ia: 1 for the rest velocity, else -|c_ia - c_ia c_i^2 / 2| */
static double Bcoef(int i, int a)
{
    int c2 = CX[i] * CX[i] + CY[i] * CY[i];
    if (c2 == 0) return 1.0;
    double ca = a == 0 ? CX[i] : CY[i];
    return -fabs(ca - 0.5 * ca * c2);
}

/* A_ia = c_ia - c_ia c_i^2 / 2 (eq. Ai) */
static double Acoef(int i, int a)
{
    int c2 = CX[i] * CX[i] + CY[i] * CY[i];
    double ca = a == 0 ? CX[i] : CY[i];
    return ca - 0.5 * ca * c2;
}

static void geq_parts(double rho, double ux, double uy, double T, double E,
                      double *qeq, double *Req, double *psi)
{
    double u[2] = {ux, uy};
    /* q^eq_a = 2 rho u_a (E + T) */
    qeq[0] = 2.0 * rho * ux * (E + T);
    qeq[1] = 2.0 * rho * uy * (E + T);
    /* R^eq_ab = 2 rho E (T d_ab + u_a u_b) + 2 rho T (T d_ab + 2 u_a u_b) */
    Req[0] = 2.0 * rho * E * (T + ux * ux) + 2.0 * rho * T * (T + 2.0 * ux * ux);
    Req[1] = 2.0 * rho * E * (ux * uy) + 2.0 * rho * T * (2.0 * ux * uy);
    Req[2] = 2.0 * rho * E * (T + uy * uy) + 2.0 * rho * T * (T + 2.0 * uy * uy);
    /* psi_i = B_ia rho (1 - 3T)(T^2 + 2 u_a^2 T + E u_a^2) / T */
    double Z[2];
    for (int a = 0; a < 2; ++a)
        Z[a] = rho * (1.0 - 3.0 * T) * (T * T + 2.0 * u[a] * u[a] * T + E * u[a] * u[a]) / T;
    for (int i = 0; i < Q; ++i) psi[i] = Bcoef(i, 0) * Z[0] + Bcoef(i, 1) * Z[1];
}

void orc_geq(double rho, double ux, double uy, double T, double gamma, double *g)
{
    double Cv = 1.0 / (gamma - 1.0);
    double E = Cv * T + 0.5 * (ux * ux + uy * uy);
    double qeq[2], Req[3], psi[Q];
    geq_parts(rho, ux, uy, T, E, qeq, Req, psi);
    Gform(T, 2.0 * rho * E, qeq, Req, psi, g);
}

/* quasi-equilibrium g* with q*_a = q^eq_a + 2 u_b (P_ab - P^eq_ab) (tab. Eq_Moments;
   the q^eq term restores g* = g^eq at equilibrium) ; P = {xx, xy, yy} */
void orc_gqe(double rho, double ux, double uy, double T, double gamma, const double *P, double *g)
{
    double Cv = 1.0 / (gamma - 1.0);
    double E = Cv * T + 0.5 * (ux * ux + uy * uy);
    double qeq[2], Req[3], psi[Q];
    geq_parts(rho, ux, uy, T, E, qeq, Req, psi);
    double Peq[3] = {rho * ux * ux + rho * T, rho * ux * uy, rho * uy * uy + rho * T};
    double dP[3] = {P[0] - Peq[0], P[1] - Peq[1], P[2] - Peq[2]};
    double qs[2];
    qs[0] = qeq[0] + 2.0 * (ux * dP[0] + uy * dP[1]);
    qs[1] = qeq[1] + 2.0 * (ux * dP[1] + uy * dP[2]);
    Gform(T, 2.0 * rho * E, qs, Req, psi, g);
}

/* moments of streamed populations (Sec. IV conservation constraints, eq. Temp) */
static void moments(const double *ft, const double *gt, double Cv, double *rho, double *ux,
                    double *uy, double *E, double *T, double *P)
{
    double r = 0, jx = 0, jy = 0, s = 0, pxx = 0, pxy = 0, pyy = 0;
    for (int i = 0; i < Q; ++i) {
        r += ft[i];
        jx += CX[i] * ft[i];
        jy += CY[i] * ft[i];
        pxx += CX[i] * CX[i] * ft[i];
        pxy += CX[i] * CY[i] * ft[i];
        pyy += CY[i] * CY[i] * ft[i];
        s += gt[i];
    }
    *rho = r;
    *ux = jx / r;
    *uy = jy / r;
    *E = s / (2.0 * r);
    *T = (*E - 0.5 * ((*ux) * (*ux) + (*uy) * (*uy))) / Cv;
    if (P) { P[0] = pxx; P[1] = pxy; P[2] = pyy; }
}

/* collision (eqs. feqn, geqn) with phi_i = A_ia X_a */
void orc_collide(const double *ft, const double *gt, const double *Xa, double gamma, double Pr,
                 double mu, double dt, double *fs, double *gs)
{
    double Cv = 1.0 / (gamma - 1.0);
    double rho, ux, uy, E, T, P[3];
    moments(ft, gt, Cv, &rho, &ux, &uy, &E, &T, P);
    /* mu = (1/w - 1/2) rho T dt ; kappa = Cp (1/w1 - 1/2) rho T dt, Pr = Cp mu / kappa */
    double om = 1.0 / (mu / (rho * T * dt) + 0.5);
    double om1 = 1.0 / (mu / (Pr * rho * T * dt) + 0.5);
    double feq[Q], geq[Q], gqe[Q];
    orc_feq(rho, ux, uy, T, feq);
    orc_geq(rho, ux, uy, T, gamma, geq);
    orc_gqe(rho, ux, uy, T, gamma, P, gqe);
    for (int i = 0; i < Q; ++i) {
        double phi = Acoef(i, 0) * Xa[0] + Acoef(i, 1) * Xa[1];
        fs[i] = ft[i] + om * (feq[i] - ft[i]) + dt * phi;
        gs[i] = gt[i] + om * (geq[i] - gt[i]) + (om1 - om) * (gqe[i] - gt[i]);
    }
}

/* Grad approximation of missing populations (Sec. IV.A, tab. Neq_Moments):
 *   f^miss = f^eq + dt f^(1), g^miss = g^eq + dt g^(1)
 * gradu = {du_x/dx, du_x/dy, du_y/dx, du_y/dy}, gradT = {dT/dx, dT/dy} (physical) */
void orc_grad_missing(double rho, double ux, double uy, double T, const double *gradu,
                      const double *gradT, double gamma, double Pr, double mu, double dt,
                      double *fm, double *gm)
{
    double Cv = 1.0 / (gamma - 1.0), Cp = Cv + 1.0;
    double E = Cv * T + 0.5 * (ux * ux + uy * uy);
    double om = 1.0 / (mu / (rho * T * dt) + 0.5);
    double om1 = 1.0 / (mu / (Pr * rho * T * dt) + 0.5);
    double u[2] = {ux, uy};
    /* du[a][b] = d_a u_b */
    double du[2][2] = {{gradu[0], gradu[2]}, {gradu[1], gradu[3]}};
    double S[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) S[a][b] = du[a][b] + du[b][a];
    double divu = du[0][0] + du[1][1];
    double dE[2];
    for (int a = 0; a < 2; ++a) dE[a] = Cv * gradT[a] + u[0] * du[a][0] + u[1] * du[a][1];
    double P1[2][2], R1[2][2], q1[2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            P1[a][b] = -(1.0 / om) * rho * T * (S[a][b] - (a == b ? divu / Cv : 0.0));
        }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            R1[a][b] = -(2.0 / om1) * rho * T * (S[a][b] * (E + 2.0 * T) + u[a] * dE[b] + u[b] * dE[a]);
    for (int a = 0; a < 2; ++a)
        q1[a] = -(2.0 / om1) * rho * Cp * T * gradT[a] + 2.0 * (u[0] * P1[a][0] + u[1] * P1[a][1]);
    double feq[Q], geq[Q], f1[Q], g1[Q];
    orc_feq(rho, ux, uy, T, feq);
    orc_geq(rho, ux, uy, T, gamma, geq);
    double zero2[2] = {0.0, 0.0};
    double P1v[3] = {P1[0][0], P1[0][1], P1[1][1]};
    double R1v[3] = {R1[0][0], R1[0][1], R1[1][1]};
    Gform(T, 0.0, zero2, P1v, NULL, f1);
    Gform(T, 0.0, q1, R1v, NULL, g1);
    for (int i = 0; i < Q; ++i) {
        fm[i] = feq[i] + dt * f1[i];
        gm[i] = geq[i] + dt * g1[i];
    }
}

/* ------------------------------------------------------------------------ */
/* set-up                                                                   */
/* ------------------------------------------------------------------------ */
static double min_image(double p, double ref, double L)
{
    if (L <= 0.0) return p;
    return p + L * nearbyint((ref - p) / L);
}

orc_t *orc_create(int32_t nn, int32_t ne, int32_t nv, const double *X, const int32_t *elem, const int32_t *nbr,
                  const int8_t *pshift, const double *period, int32_t nwe, const int32_t *wall_edges,
                  const orc_params_t *p, int32_t *status)
{
    *status = ORC_OK;
    orc_t *o = (orc_t *)calloc(1, sizeof(orc_t));
    o->nn = nn; o->ne = ne; o->nwe = nwe;
    if (nv != 6 && nv != 9) {
        snprintf(o->err, sizeof o->err, "elements have 6 (P2 triangle) or 9 (Q2 quadrilateral) nodes, not %d", nv);
        *status = ORC_EINVAL;
        return o;
    }
    o->kind = nv == 9;
    o->nv = nv;
    o->nf = nv == 9 ? 4 : 3;
    const int NV = o->nv, NF = o->nf;
    o->p = *p;
    o->Cv = 1.0 / (p->gamma - 1.0);
    o->Cp = o->Cv + 1.0;
    o->period[0] = period ? period[0] : 0.0;
    o->period[1] = period ? period[1] : 0.0;
    o->X = (double *)malloc(sizeof(double) * 2 * nn);
    memcpy(o->X, X, sizeof(double) * 2 * nn);
    o->elem = (int *)malloc(sizeof(int) * NV * ne);
    memcpy(o->elem, elem, sizeof(int) * NV * ne);
    o->nbr = (int *)malloc(sizeof(int) * NF * ne);
    memcpy(o->nbr, nbr, sizeof(int) * NF * ne);
    o->psh = (signed char *)calloc(NF * (size_t)ne, 1);
    if (pshift) memcpy(o->psh, pshift, NF * (size_t)ne);
    o->wedge = (int *)malloc(sizeof(int) * 2 * (nwe > 0 ? nwe : 1));
    if (nwe > 0) memcpy(o->wedge, wall_edges, sizeof(int) * 2 * nwe);

    /* element frames (first corner at its canonical coordinates, the others at
       their nearest periodic images), affine inverse or corners, and area */
    o->ev = (double *)malloc(sizeof(double) * 6 * ne);
    o->Ainv = (double *)malloc(sizeof(double) * 4 * ne);
    o->qc = (double *)malloc(sizeof(double) * 8 * ne);
    o->area = (double *)malloc(sizeof(double) * ne);
    for (int e = 0; e < ne; ++e) {
        const int *en = o->elem + NV * e;
        for (int k = 0; k < NV; ++k)
            if (en[k] < 0 || en[k] >= nn) {
                snprintf(o->err, sizeof o->err, "element %d references node %d out of range", e, en[k]);
                *status = ORC_EMESH;
                return o;
            }
        if (o->kind == 1) {
            double *c = o->qc + 8 * e;
            c[0] = X[2 * en[0]];
            c[1] = X[2 * en[0] + 1];
            for (int k = 1; k < 4; ++k) {
                c[2 * k] = min_image(X[2 * en[k]], c[0], o->period[0]);
                c[2 * k + 1] = min_image(X[2 * en[k] + 1], c[1], o->period[1]);
            }
            double a2 = 0.0;
            int convex = 1;
            for (int k = 0; k < 4; ++k) {
                const double *pa = c + 2 * k, *pb = c + 2 * ((k + 1) % 4), *pc = c + 2 * ((k + 2) % 4);
                a2 += pa[0] * pb[1] - pa[1] * pb[0];
                if ((pb[0] - pa[0]) * (pc[1] - pb[1]) - (pb[1] - pa[1]) * (pc[0] - pb[0]) <= 0.0) convex = 0;
            }
            o->area[e] = 0.5 * a2;
            if (!convex) {
                snprintf(o->err, sizeof o->err, "quadrilateral %d is not strictly convex and counter-clockwise", e);
                *status = ORC_EMESH;
                return o;
            }
            continue;
        }
        double *v = o->ev + 6 * e;
        v[0] = X[2 * en[0]];
        v[1] = X[2 * en[0] + 1];
        for (int k = 1; k < 3; ++k) {
            v[2 * k] = min_image(X[2 * en[k]], v[0], o->period[0]);
            v[2 * k + 1] = min_image(X[2 * en[k] + 1], v[1], o->period[1]);
        }
        double b00 = v[2] - v[0], b01 = v[4] - v[0], b10 = v[3] - v[1], b11 = v[5] - v[1];
        double det = b00 * b11 - b01 * b10;
        o->area[e] = 0.5 * det;
        if (!(det > 0.0)) {
            snprintf(o->err, sizeof o->err, "element %d has non-positive area", e);
            *status = ORC_EMESH;
            return o;
        }
        double *A = o->Ainv + 4 * e;
        A[0] = b11 / det;  A[1] = -b01 / det;
        A[2] = -b10 / det; A[3] = b00 / det;
    }
    /* neighbour symmetry */
    for (int e = 0; e < ne; ++e)
        for (int k = 0; k < NF; ++k) {
            int n = o->nbr[NF * e + k];
            if (n >= ne || n < -2) {
                snprintf(o->err, sizeof o->err, "neighbour of element %d out of range", e);
                *status = ORC_EMESH;
                return o;
            }
            int back = 0;
            for (int j = 0; n >= 0 && j < NF; ++j) back |= o->nbr[NF * n + j] == e;
            if (n >= 0 && !back) {
                snprintf(o->err, sizeof o->err, "neighbours of elements %d and %d are not symmetric", e, n);
                *status = ORC_EMESH;
                return o;
            }
        }
    /* owner element: the containing element of largest (computational) area,
       ties to the lowest element index (Sec. IV, last paragraph before IV.A) */
    o->owner = (int *)malloc(sizeof(int) * nn);
    o->oslot = (int *)malloc(sizeof(int) * nn);
    o->opos = (double *)malloc(sizeof(double) * 2 * nn);
    for (int a = 0; a < nn; ++a) o->owner[a] = -1;
    for (int e = 0; e < ne; ++e)
        for (int k = 0; k < NV; ++k) {
            int a = o->elem[NV * e + k];
            int cur = o->owner[a];
            if (cur < 0 || o->area[e] > o->area[cur]) {
                o->owner[a] = e;
                o->oslot[a] = k;
            }
        }
    for (int a = 0; a < nn; ++a) {
        if (o->owner[a] < 0) {
            snprintf(o->err, sizeof o->err, "node %d belongs to no element", a);
            *status = ORC_EMESH;
            return o;
        }
        elem_node_pos(o, o->owner[a], o->oslot[a], o->opos + 2 * a);
    }
    /* wall nodes, their computational into-fluid normals and point B (Sec. IV.A) */
    o->wid = (int *)malloc(sizeof(int) * nn);
    for (int a = 0; a < nn; ++a) o->wid[a] = -1;
    double *nacc = (double *)calloc(2 * (size_t)nn, sizeof(double));
    int nw = 0;
    for (int w = 0; w < nwe; ++w) {
        int e = o->wedge[2 * w], k = o->wedge[2 * w + 1];
        if (e < 0 || e >= ne || k < 0 || k >= NF || o->nbr[NF * e + k] != -1) {
            snprintf(o->err, sizeof o->err, "wall edge %d is not a wall-tagged element edge", w);
            *status = ORC_EMESH;
            free(nacc);
            return o;
        }
        int slots[3];
        double pa[2], pb[2];
        elem_edge(o, e, k, slots, pa, pb);
        double dx = pb[0] - pa[0], dy = pb[1] - pa[1];
        double L = sqrt(dx * dx + dy * dy);
        double nx = -dy / L, ny = dx / L; /* into the (counter-clockwise) element */
        int nodes[3] = {o->elem[NV * e + slots[0]], o->elem[NV * e + slots[2]], o->elem[NV * e + slots[1]]};
        for (int j = 0; j < 3; ++j) {
            int a = nodes[j];
            if (o->wid[a] < 0) o->wid[a] = nw++;
            nacc[2 * a] += nx;
            nacc[2 * a + 1] += ny;
        }
    }
    o->nw = nw;
    o->wnorm = (double *)malloc(sizeof(double) * 2 * (nw > 0 ? nw : 1));
    o->bel = (int *)malloc(sizeof(int) * (nw > 0 ? nw : 1));
    o->blam = (double *)malloc(sizeof(double) * 3 * (nw > 0 ? nw : 1));
    for (int a = 0; a < nn; ++a) {
        int w = o->wid[a];
        if (w < 0) continue;
        double L = sqrt(nacc[2 * a] * nacc[2 * a] + nacc[2 * a + 1] * nacc[2 * a + 1]);
        o->wnorm[2 * w] = nacc[2 * a] / L;
        o->wnorm[2 * w + 1] = nacc[2 * a + 1] / L;
        /* B = A + dt n, located once (the computational mesh is fixed) */
        double B[2] = {o->opos[2 * a] + p->dt * o->wnorm[2 * w], o->opos[2 * a + 1] + p->dt * o->wnorm[2 * w + 1]};
        int eb;
        double lam[3];
        int st = orc_locate(o, o->owner[a], B, &eb, lam, NULL);
        if (st != 0) {
            snprintf(o->err, sizeof o->err, "point B of wall node %d lies outside the mesh", a);
            *status = ORC_EMESH;
            free(nacc);
            return o;
        }
        o->bel[w] = eb;
        o->blam[3 * w] = lam[0]; o->blam[3 * w + 1] = lam[1]; o->blam[3 * w + 2] = lam[2];
    }
    free(nacc);

    size_t n9 = (size_t)nn * Q;
    o->f = (double *)calloc(n9, sizeof(double));
    o->g = (double *)calloc(n9, sizeof(double));
    o->ft = (double *)calloc(n9, sizeof(double));
    o->gt = (double *)calloc(n9, sizeof(double));
    o->M = (double *)calloc(4 * (size_t)nn, sizeof(double));
    o->Mn = (double *)calloc(4 * (size_t)nn, sizeof(double));
    o->W = (double *)calloc(2 * (size_t)nn, sizeof(double));
    o->Xa = (double *)calloc(2 * (size_t)nn, sizeof(double));
    o->mw = (int *)calloc(nn, sizeof(int));
    o->mf = (int *)calloc(nn, sizeof(int));
    o->t = p->t0;
    o->step = 0;
    return o;
}

void orc_destroy(orc_t *o)
{
    if (!o) return;
    free(o->X); free(o->elem); free(o->nbr); free(o->psh); free(o->wedge);
    free(o->ev); free(o->Ainv); free(o->qc); free(o->area); free(o->owner); free(o->oslot); free(o->opos);
    free(o->wid); free(o->wnorm); free(o->bel); free(o->blam);
    free(o->f); free(o->g); free(o->ft); free(o->gt); free(o->M); free(o->Mn);
    free(o->W); free(o->Xa); free(o->mw); free(o->mf);
    free(o);
}

const char *orc_error(const orc_t *o) { return o ? o->err : "null handle"; }

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* threads of the parallel loops from now on (timing only: every loop is over
   independent nodes, so the results do not depend on it) */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* initial condition: f = f^eq, g = g^eq of the given fields */
int orc_init_fields(orc_t *o, const double *rho, const double *ux, const double *uy, const double *T)
{
    for (int a = 0; a < o->nn; ++a) {
        orc_feq(rho[a], ux[a], uy[a], T[a], o->f + Q * (size_t)a);
        orc_geq(rho[a], ux[a], uy[a], T[a], o->p.gamma, o->g + Q * (size_t)a);
        o->M[4 * a] = rho[a]; o->M[4 * a + 1] = ux[a]; o->M[4 * a + 2] = uy[a]; o->M[4 * a + 3] = T[a];
    }
    o->step = 0;
    o->t = o->p.t0;
    return ORC_OK;
}

/* gradient of a nodal field at node a through its owner element, in computational coordinates */
static void owner_grad(const orc_t *o, int a, const double *K, int stride, int comp, double *gX)
{
    int e = o->owner[a];
    double gN[9][2];
    elem_grad_slot(o, e, o->oslot[a], gN);
    gX[0] = gX[1] = 0.0;
    for (int s = 0; s < o->nv; ++s) {
        double k = K[(size_t)stride * o->elem[o->nv * e + s] + comp];
        gX[0] += k * gN[s][0];
        gX[1] += k * gN[s][1];
    }
}

/* ------------------------------------------------------------------------ */
/* one time step                                                            */
/* ------------------------------------------------------------------------ */
static int one_step(orc_t *o)
{
    const orc_params_t *p = &o->p;
    const double dt = p->dt, Cv = o->Cv;
    const double th = o->t + 0.5 * dt, t1 = o->t + dt;
    int status = ORC_OK;

    /* steps 1-5: departure, locate, interpolate, missing populations */
#pragma omp parallel for schedule(static) reduction(min : status)
    for (int a = 0; a < o->nn; ++a) {
        double Xa = o->X[2 * a], Ya = o->X[2 * a + 1];
        double x[2], J[4], v[2], Ji[4], det;
        int mw = 0, mf = 0;
        for (int i = 0; i < Q; ++i) {
            /* c^_i = J^-1 (c_i - v_g) at the arrival node, then at the midpoint
               of the backward trajectory (both at t^{n+1/2}) */
            orc_motion(p, Xa, Ya, th, x, J, v);
            if (inv2(J, Ji, &det) != 0) { status = ORC_EJAC; break; }
            double wx = CX[i] - v[0], wy = CY[i] - v[1];
            double chx = Ji[0] * wx + Ji[1] * wy, chy = Ji[2] * wx + Ji[3] * wy;
            double Xm = Xa - 0.5 * dt * chx, Ym = Ya - 0.5 * dt * chy;
            orc_motion(p, Xm, Ym, th, x, J, v);
            if (inv2(J, Ji, &det) != 0) { status = ORC_EJAC; break; }
            wx = CX[i] - v[0]; wy = CY[i] - v[1];
            chx = Ji[0] * wx + Ji[1] * wy;
            chy = Ji[2] * wx + Ji[3] * wy;
            /* departure point in the owner element's frame */
            double P[2] = {o->opos[2 * a] - dt * chx, o->opos[2 * a + 1] - dt * chy};
            int e;
            double l[3], N[9];
            int st = orc_locate(o, o->owner[a], P, &e, l, NULL);
            if (st == ORC_ELOCATE) { status = ORC_ELOCATE; break; }
            if (st == -1) { mw |= 1 << i; continue; }
            if (st == -2) { mf |= 1 << i; continue; }
            elem_shape(o, l, N);
            double sf = 0.0, sg = 0.0;
            for (int s = 0; s < o->nv; ++s) {
                int b = o->elem[o->nv * e + s];
                sf += N[s] * o->f[Q * (size_t)b + i];
                sg += N[s] * o->g[Q * (size_t)b + i];
            }
            o->ft[Q * (size_t)a + i] = sf;
            o->gt[Q * (size_t)a + i] = sg;
        }
        o->mw[a] = mw;
        o->mf[a] = mf;
        if (mf) {
            /* far field: free-stream equilibrium */
            double fe[Q], ge[Q];
            orc_feq(p->rho_inf, p->u_inf[0], p->u_inf[1], p->T_inf, fe);
            orc_geq(p->rho_inf, p->u_inf[0], p->u_inf[1], p->T_inf, p->gamma, ge);
            for (int i = 0; i < Q; ++i)
                if (mf & (1 << i)) {
                    o->ft[Q * (size_t)a + i] = fe[i];
                    o->gt[Q * (size_t)a + i] = ge[i];
                }
        }
        if (mw) {
            /* targets: wall node -> wall velocity, rho and T at B; other node ->
               its own values of the previous step */
            double rt, ut[2], Tt;
            int w = o->wid[a];
            if (w >= 0) {
                orc_motion(p, Xa, Ya, t1, x, J, v);
                ut[0] = v[0]; ut[1] = v[1];
                double N[9];
                elem_shape(o, o->blam + 3 * w, N);
                rt = 0.0; Tt = 0.0;
                for (int s = 0; s < o->nv; ++s) {
                    int b = o->elem[o->nv * o->bel[w] + s];
                    rt += N[s] * o->M[4 * (size_t)b];
                    Tt += N[s] * o->M[4 * (size_t)b + 3];
                }
            } else {
                rt = o->M[4 * (size_t)a];
                ut[0] = o->M[4 * (size_t)a + 1];
                ut[1] = o->M[4 * (size_t)a + 2];
                Tt = o->M[4 * (size_t)a + 3];
            }
            /* gradients of the previous-step u and T at the node, physical, at t^{n+1} */
            double gX[2], gux[2] = {0, 0}, guy[2] = {0, 0}, gT[2] = {0, 0};
            owner_grad(o, a, o->M, 4, 1, gX);
            if (phys_grad(p, Xa, Ya, t1, gX, gux) != 0) status = ORC_EJAC;
            owner_grad(o, a, o->M, 4, 2, gX);
            phys_grad(p, Xa, Ya, t1, gX, guy);
            owner_grad(o, a, o->M, 4, 3, gX);
            phys_grad(p, Xa, Ya, t1, gX, gT);
            double gradu[4] = {gux[0], gux[1], guy[0], guy[1]};
            double fm[Q], gm[Q];
            orc_grad_missing(rt, ut[0], ut[1], Tt, gradu, gT, p->gamma, p->Pr, p->mu, dt, fm, gm);
            for (int i = 0; i < Q; ++i)
                if (mw & (1 << i)) {
                    o->ft[Q * (size_t)a + i] = fm[i];
                    o->gt[Q * (size_t)a + i] = gm[i];
                }
        }
    }
    if (status != ORC_OK) {
        snprintf(o->err, sizeof o->err, "step %ld: %s", o->step,
                 status == ORC_EJAC ? "non-positive mapping Jacobian" : "walk exceeded its step cap");
        return status;
    }

    /* step 6: moments */
#pragma omp parallel for schedule(static)
    for (int a = 0; a < o->nn; ++a) {
        double rho, ux, uy, E, T;
        moments(o->ft + Q * (size_t)a, o->gt + Q * (size_t)a, Cv, &rho, &ux, &uy, &E, &T, NULL);
        o->Mn[4 * (size_t)a] = rho;
        o->Mn[4 * (size_t)a + 1] = ux;
        o->Mn[4 * (size_t)a + 2] = uy;
        o->Mn[4 * (size_t)a + 3] = T;
    }

    if (!(p->flags & ORC_F_NO_COLLIDE)) {
        /* step 7: W_a = (mu / rho T) d_a Q'_aaa, Q'_aaa = rho u_a (1 - 3T) - rho u_a^3 */
        double *Qp = (double *)malloc(sizeof(double) * 2 * (size_t)o->nn);
#pragma omp parallel for schedule(static)
        for (int a = 0; a < o->nn; ++a) {
            double rho = o->Mn[4 * (size_t)a], T = o->Mn[4 * (size_t)a + 3];
            for (int d = 0; d < 2; ++d) {
                double u = o->Mn[4 * (size_t)a + 1 + d];
                Qp[2 * (size_t)a + d] = rho * u * (1.0 - 3.0 * T) - rho * u * u * u;
            }
        }
#pragma omp parallel for schedule(static)
        for (int a = 0; a < o->nn; ++a) {
            double gX[2], gx[2] = {0, 0};
            double rho = o->Mn[4 * (size_t)a], T = o->Mn[4 * (size_t)a + 3];
            for (int d = 0; d < 2; ++d) {
                owner_grad(o, a, Qp, 2, d, gX);
                phys_grad(p, o->X[2 * a], o->X[2 * a + 1], t1, gX, gx);
                o->W[2 * (size_t)a + d] = p->mu / (rho * T) * gx[d];
            }
        }
        free(Qp);
        /* step 8: X_a = - d_a W_a */
#pragma omp parallel for schedule(static)
        for (int a = 0; a < o->nn; ++a) {
            double gX[2], gx[2] = {0, 0};
            for (int d = 0; d < 2; ++d) {
                owner_grad(o, a, o->W, 2, d, gX);
                phys_grad(p, o->X[2 * a], o->X[2 * a + 1], t1, gX, gx);
                o->Xa[2 * (size_t)a + d] = -gx[d];
            }
        }
        /* step 9: collision */
        int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
        for (int a = 0; a < o->nn; ++a) {
            orc_collide(o->ft + Q * (size_t)a, o->gt + Q * (size_t)a, o->Xa + 2 * (size_t)a, p->gamma,
                        p->Pr, p->mu, dt, o->f + Q * (size_t)a, o->g + Q * (size_t)a);
            if (p->flags & ORC_F_CHECK_FINITE)
                for (int i = 0; i < Q; ++i)
                    if (!isfinite(o->f[Q * (size_t)a + i]) || !isfinite(o->g[Q * (size_t)a + i])) bad = 1;
        }
        if (bad) {
            snprintf(o->err, sizeof o->err, "step %ld: non-finite populations", o->step);
            status = ORC_ENONFINITE;
        }
    } else {
        memcpy(o->f, o->ft, sizeof(double) * Q * (size_t)o->nn);
        memcpy(o->g, o->gt, sizeof(double) * Q * (size_t)o->nn);
    }
    memcpy(o->M, o->Mn, sizeof(double) * 4 * (size_t)o->nn);
    o->t = t1;
    o->step += 1;
    return status;
}

int orc_step(orc_t *o, int32_t n)
{
    for (int s = 0; s < n; ++s) {
        int st = one_step(o);
        if (st != ORC_OK) return st;
    }
    return ORC_OK;
}

int orc_get_state(const orc_t *o, double *pops, double *macros, double *t, int64_t *step)
{
    size_t N = o->nn;
    for (size_t a = 0; a < N; ++a) {
        for (int i = 0; i < Q; ++i) {
            if (pops) {
                pops[i * N + a] = o->f[Q * a + i];
                pops[(Q + i) * N + a] = o->g[Q * a + i];
            }
        }
        if (macros)
            for (int k = 0; k < 4; ++k) macros[k * N + a] = o->M[4 * a + k];
    }
    if (t) *t = o->t;
    if (step) *step = o->step;
    return ORC_OK;
}

int orc_set_state(orc_t *o, const double *pops, const double *macros, double t, int64_t step)
{
    size_t N = o->nn;
    for (size_t a = 0; a < N; ++a) {
        for (int i = 0; i < Q; ++i) {
            o->f[Q * a + i] = pops[i * N + a];
            o->g[Q * a + i] = pops[(Q + i) * N + a];
        }
        for (int k = 0; k < 4; ++k) o->M[4 * a + k] = macros[k * N + a];
    }
    o->t = t;
    o->step = step;
    return ORC_OK;
}

int orc_get_streamed(const orc_t *o, double *pops, int32_t *miss_wall, int32_t *miss_far)
{
    size_t N = o->nn;
    for (size_t a = 0; a < N; ++a) {
        if (pops)
            for (int i = 0; i < Q; ++i) {
                pops[i * N + a] = o->ft[Q * a + i];
                pops[(Q + i) * N + a] = o->gt[Q * a + i];
            }
        if (miss_wall) miss_wall[a] = o->mw[a];
        if (miss_far) miss_far[a] = o->mf[a];
    }
    return ORC_OK;
}

int orc_get_correction(const orc_t *o, double *W, double *Xa)
{
    size_t N = o->nn;
    for (size_t a = 0; a < N; ++a)
        for (int d = 0; d < 2; ++d) {
            if (W) W[d * N + a] = o->W[2 * a + d];
            if (Xa) Xa[d * N + a] = o->Xa[2 * a + d];
        }
    return ORC_OK;
}

int orc_get_owner(const orc_t *o, int32_t *owner)
{
    for (int a = 0; a < o->nn; ++a) owner[a] = o->owner[a];
    return ORC_OK;
}

int orc_move_mesh(const orc_t *o, double t, double *x, double *Jinv, double *detJ, double *vg)
{
    int st = ORC_OK;
    for (int a = 0; a < o->nn; ++a) {
        double xx[2], J[4], v[2], Ji[4] = {0, 0, 0, 0}, det = 0.0;
        orc_motion(&o->p, o->X[2 * a], o->X[2 * a + 1], t, xx, J, v);
        if (inv2(J, Ji, &det) != 0) st = ORC_EJAC;
        if (x) { x[2 * a] = xx[0]; x[2 * a + 1] = xx[1]; }
        if (Jinv) for (int k = 0; k < 4; ++k) Jinv[4 * a + k] = Ji[k];
        if (detJ) detJ[a] = det;
        if (vg) { vg[2 * a] = v[0]; vg[2 * a + 1] = v[1]; }
    }
    return st;
}

int orc_node_gradient(const orc_t *o, const double *K, double t, double *grad)
{
    int st = ORC_OK;
    for (int a = 0; a < o->nn; ++a) {
        double gX[2], gx[2] = {0, 0};
        owner_grad(o, a, K, 1, 0, gX);
        if (phys_grad(&o->p, o->X[2 * a], o->X[2 * a + 1], t, gX, gx) != 0) st = ORC_EJAC;
        grad[2 * a] = gx[0];
        grad[2 * a + 1] = gx[1];
    }
    return st;
}

int orc_interpolate(const orc_t *o, int32_t e, const double *P, const double *K, double *val)
{
    int eo;
    double l[3], N[9];
    int st = orc_locate(o, e, P, &eo, l, NULL);
    if (st != 0) return st;
    elem_shape(o, l, N);
    double s = 0.0;
    for (int k = 0; k < o->nv; ++k) s += N[k] * K[o->elem[o->nv * eo + k]];
    *val = s;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* force on the walls at the current time (coefficients of Sec. V.B, V.C):
 * traction sigma n on straight wall edges (3 nodes each), Simpson weights
 * 1/6, 4/6, 1/6;
 * p = rho T, viscous stress mu (S - (1/Cv) div u I) with gradients from the
 * wall edge's own element                                                   */
/* ------------------------------------------------------------------------ */
int orc_forces(const orc_t *o, double *out)
{
    const orc_params_t *p = &o->p;
    double t = o->t;
    double Fp[2] = {0, 0}, Fv[2] = {0, 0}, Mp = 0.0, Mv = 0.0;
    for (int w = 0; w < o->nwe; ++w) {
        int e = o->wedge[2 * w], k = o->wedge[2 * w + 1];
        int slots[3];
        double ca[2], cb[2];
        elem_edge(o, e, k, slots, ca, cb);
        double xa[2], xb[2], J[4], vv[2];
        orc_motion(p, ca[0], ca[1], t, xa, J, vv);
        orc_motion(p, cb[0], cb[1], t, xb, J, vv);
        double dx = xb[0] - xa[0], dy = xb[1] - xa[1];
        double len = sqrt(dx * dx + dy * dy);
        /* normal out of the body (into the fluid element) */
        double nx = -dy / len, ny = dx / len;
        double wts[3] = {1.0 / 6.0, 4.0 / 6.0, 1.0 / 6.0};
        for (int j = 0; j < 3; ++j) {
            int s = slots[j];
            int a = o->elem[o->nv * e + s];
            double gN[9][2], pos[2];
            elem_grad_slot(o, e, s, gN);
            elem_node_pos(o, e, s, pos);
            double X0 = pos[0], Y0 = pos[1];
            double gu[2][2]; /* gu[c][d] = d u_c / d x_d */
            for (int c = 0; c < 2; ++c) {
                double gX[2] = {0, 0};
                for (int q = 0; q < o->nv; ++q) {
                    double uq = o->M[4 * (size_t)o->elem[o->nv * e + q] + 1 + c];
                    gX[0] += uq * gN[q][0];
                    gX[1] += uq * gN[q][1];
                }
                phys_grad(p, X0, Y0, t, gX, gu[c]);
            }
            double divu = gu[0][0] + gu[1][1];
            double tau[2][2];
            for (int c = 0; c < 2; ++c)
                for (int d = 0; d < 2; ++d)
                    tau[c][d] = p->mu * (gu[c][d] + gu[d][c] - (c == d ? divu / o->Cv : 0.0));
            double pr = o->M[4 * (size_t)a] * o->M[4 * (size_t)a + 3];
            double xn[2], Jn[4], vn[2];
            orc_motion(p, X0, Y0, t, xn, Jn, vn);
            double rx = xn[0] - p->ref_point[0], ry = xn[1] - p->ref_point[1];
            double tp[2] = {-pr * nx, -pr * ny};
            double tv[2] = {tau[0][0] * nx + tau[0][1] * ny, tau[1][0] * nx + tau[1][1] * ny};
            double wl = wts[j] * len;
            Fp[0] += wl * tp[0]; Fp[1] += wl * tp[1];
            Fv[0] += wl * tv[0]; Fv[1] += wl * tv[1];
            /* nose-up positive: minus the z component of r x traction */
            Mp += -wl * (rx * tp[1] - ry * tp[0]);
            Mv += -wl * (rx * tv[1] - ry * tv[0]);
        }
    }
    double U2 = p->u_inf[0] * p->u_inf[0] + p->u_inf[1] * p->u_inf[1];
    double qc = 0.5 * p->rho_inf * U2 * p->chord;
    out[0] = Fp[0]; out[1] = Fp[1]; out[2] = Fv[0]; out[3] = Fv[1];
    out[4] = Mp; out[5] = Mv;
    out[6] = qc > 0 ? (Fp[1] + Fv[1]) / qc : 0.0;
    out[7] = qc > 0 ? (Fp[0] + Fv[0]) / qc : 0.0;
    out[8] = qc > 0 ? (Mp + Mv) / (qc * p->chord) : 0.0;
    out[9] = t;
    return ORC_OK;
}
