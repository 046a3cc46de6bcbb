// Host runtime of the ALE lattice-Boltzmann library: the C-ABI declared in
// include/alelb.h.  Builds the static mesh data of every case (element frames
// and affine inverses, owner map, wall normals and points B), reorders each
// case's nodes and elements along a Hilbert curve, concatenates the cases into
// one set of device arrays, owns the device buffers and enqueues the gfx950
// kernels of alelb_kernels.hip on the caller's stream (optionally as a HIP
// graph of two steps).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

#include "alelb.h"
#include "alelb_impl.h"

using namespace alelb;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_OK(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(e_ == hipErrorOutOfMemory ? ALE_LB_ENOMEM : ALE_LB_EDEVICE, "%s: %s", \
                        #expr, hipGetErrorString(e_));                                      \
    } while (0)

double min_image(double p, double ref, double L)
{
    return L > 0.0 ? p + L * std::nearbyint((ref - p) / L) : p;
}

// Index along a Hilbert curve of order 21 of the cell (x, y), 0 <= x, y < 2^21:
// quadrant by quadrant from the coarsest level, each step rotating or
// reflecting the remaining coordinates into the sub-square's own orientation.
// Unlike a Morton key, consecutive indices are always adjacent cells.
uint64_t hilbert_index(uint64_t x, uint64_t y)
{
    const uint64_t n = uint64_t(1) << 21;
    uint64_t d = 0;
    for (uint64_t s = n >> 1; s > 0; s >>= 1) {
        const uint64_t rx = (x & s) ? 1 : 0, ry = (y & s) ? 1 : 0;
        d += s * s * ((3 * rx) ^ ry);
        if (ry == 0) {
            if (rx == 1) {
                x = n - 1 - x;
                y = n - 1 - y;
            }
            std::swap(x, y);
        }
    }
    return d;
}

// Hilbert order of a point set over its bounding box (ties by index)
std::vector<int> hilbert_order(const std::vector<double> &xy)
{
    const size_t n = xy.size() / 2;
    double lo[2] = {1e300, 1e300}, hi[2] = {-1e300, -1e300};
    for (size_t i = 0; i < n; ++i)
        for (int d = 0; d < 2; ++d) {
            lo[d] = std::min(lo[d], xy[2 * i + d]);
            hi[d] = std::max(hi[d], xy[2 * i + d]);
        }
    const double ext = std::max(std::max(hi[0] - lo[0], hi[1] - lo[1]), 1e-300);
    std::vector<uint64_t> key(n);
    for (size_t i = 0; i < n; ++i) {
        const uint64_t qx = uint64_t(std::min(2097151.0, (xy[2 * i] - lo[0]) / ext * 2097151.0));
        const uint64_t qy = uint64_t(std::min(2097151.0, (xy[2 * i + 1] - lo[1]) / ext * 2097151.0));
        key[i] = hilbert_index(qx, qy);
    }
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return key[a] < key[b]; });
    return ord;
}

// one case's mesh: the caller's arrays and what the library derives from them
struct HostMesh {
    int N = 0, E = 0;
    int kind = ELEM_P2;
    int nv = 6, nf = 3;          // nodes and edges per element
    std::vector<double> X;       // [2N]
    std::vector<int> elem, nbr;  // [nv E], [nf E]
    std::vector<int8_t> psh;     // [nf E]
    double L[2] = {0, 0};
    std::vector<int> wedge;      // [2 NWE]
    // derived, caller order
    std::vector<double> ev;      // P2: [6E] vertex coordinates in each element frame
    std::vector<double> A;       // P2: [4E]
    std::vector<double> qc;      // Q2: [8E] corner coordinates in each element frame
    std::vector<double> area;
    std::vector<int> owner, oslot;
    std::vector<double> opos;    // [2N]
    std::vector<int> wid;        // [N] wall-node index or -1
    int nw = 0;
    std::vector<int> bel;        // [nw] element of point B (caller element index)
    std::vector<double> blam;    // [3 nw] local coordinates of B
    std::vector<int> perm, iperm, eperm, eiperm;  // Hilbert orders (internal <-> caller)
};

// local coordinates (xi, eta) of the quadrilateral nodes, as for the kernels
constexpr int QXI[9] = {-1, 1, 1, -1, 0, 1, 0, -1, 0};
constexpr int QETA[9] = {-1, -1, 1, 1, -1, 0, 1, 0, 0};

// bilinear map of corners c[8] at (xi, eta): position and Jacobian [dx/dxi dx/deta; dy/dxi dy/deta]
void q2_map_host(const double *c, double xi, double eta, double x[2], double J[4])
{
    x[0] = x[1] = J[0] = J[1] = J[2] = J[3] = 0.0;
    for (int k = 0; k < 4; ++k) {
        const double b = 0.25 * (1.0 + QXI[k] * xi) * (1.0 + QETA[k] * eta);
        const double bx = 0.25 * QXI[k] * (1.0 + QETA[k] * eta);
        const double be = 0.25 * QETA[k] * (1.0 + QXI[k] * xi);
        for (int d = 0; d < 2; ++d) {
            x[d] += b * c[2 * k + d];
            J[2 * d] += bx * c[2 * k + d];
            J[2 * d + 1] += be * c[2 * k + d];
        }
    }
}

// position of local node `slot` of element e in the element's frame
void node_pos_host(const HostMesh &h, int e, int slot, double pos[2])
{
    if (h.kind == ELEM_Q2) {
        double J[4];
        q2_map_host(&h.qc[8 * e], QXI[slot], QETA[slot], pos, J);
        return;
    }
    const double *v = &h.ev[6 * e];
    if (slot < 3) {
        pos[0] = v[2 * slot];
        pos[1] = v[2 * slot + 1];
    } else {
        const int k1 = (slot - 3 + 1) % 3, k2 = (slot - 3 + 2) % 3;
        pos[0] = 0.5 * (v[2 * k1] + v[2 * k2]);
        pos[1] = 0.5 * (v[2 * k1 + 1] + v[2 * k2 + 1]);
    }
}

// edge k of element e: its nodes (end, middle, end) counter-clockwise
void edge_slots_host(const HostMesh &h, int k, int s[3])
{
    if (h.kind == ELEM_Q2) {
        s[0] = k;
        s[1] = 4 + k;
        s[2] = (k + 1) % 4;
    } else {
        s[0] = (k + 1) % 3;
        s[1] = 3 + k;
        s[2] = (k + 2) % 3;
    }
}

// walk on the host (used once per wall node to locate its point B): the
// element holding P with P's local coordinates (barycentrics, or (xi, eta, 0)
// by Newton's method), or -1 wall, -2 far field, -4 cap
int host_walk(const HostMesh &h, int e, double P[2], double l[3])
{
    for (int it = 0; it < WALK_CAP; ++it) {
        int k = 0;
        double mn;
        if (h.kind == ELEM_Q2) {
            const double *c = &h.qc[8 * e];
            double v[4];
            for (int j = 0; j < 4; ++j) {
                const double *a = c + 2 * j, *b = c + 2 * ((j + 1) % 4);
                v[j] = (b[0] - a[0]) * (P[1] - a[1]) - (b[1] - a[1]) * (P[0] - a[0]);
            }
            mn = v[0];
            for (int j = 1; j < 4; ++j)
                if (v[j] < mn) {
                    mn = v[j];
                    k = j;
                }
            mn /= 2.0 * h.area[e];
            if (mn >= -TAU_LOC) {
                double xi = 0.0, eta = 0.0;
                for (int n = 0; n < 8; ++n) {
                    double x[2], J[4];
                    q2_map_host(c, xi, eta, x, J);
                    const double r0 = x[0] - P[0], r1 = x[1] - P[1];
                    const double det = J[0] * J[3] - J[1] * J[2];
                    const double dxi = (J[3] * r0 - J[1] * r1) / det, deta = (-J[2] * r0 + J[0] * r1) / det;
                    xi -= dxi;
                    eta -= deta;
                    if (std::fabs(dxi) + std::fabs(deta) < 1e-14) break;
                }
                l[0] = xi;
                l[1] = eta;
                l[2] = 0.0;
                return e;
            }
        } else {
            const double *v = &h.ev[6 * e];
            const double *A = &h.A[4 * e];
            const double dx = P[0] - v[0], dy = P[1] - v[1];
            l[1] = A[0] * dx + A[1] * dy;
            l[2] = A[2] * dx + A[3] * dy;
            l[0] = 1.0 - l[1] - l[2];
            mn = l[0];
            if (l[1] < mn) { k = 1; mn = l[1]; }
            if (l[2] < mn) { k = 2; mn = l[2]; }
            if (mn >= -TAU_LOC) return e;
        }
        const int n = h.nbr[h.nf * e + k];
        if (n < 0) return n;
        const int code = h.psh[h.nf * e + k];
        if (code != 0) {
            P[0] += double((code + 4) % 3 - 1) * h.L[0];
            P[1] += double((code + 4) / 3 - 1) * h.L[1];
        }
        e = n;
    }
    return -4;
}

int validate_and_derive(HostMesh &h, double dt, std::string &why)
{
    const int N = h.N, E = h.E, NV = h.nv, NF = h.nf;
    char buf[256];
    for (int e = 0; e < E; ++e)
        for (int k = 0; k < NV; ++k)
            if (h.elem[NV * e + k] < 0 || h.elem[NV * e + k] >= N) {
                snprintf(buf, sizeof buf, "element %d references node %d out of range", e, h.elem[NV * e + k]);
                why = buf;
                return ALE_LB_EMESH;
            }
    h.area.resize(E);
    if (h.kind == ELEM_Q2) {
        // corners in the element frame (corner 0 canonical, the others nearest images); strictly convex, CCW
        h.qc.resize(8 * size_t(E));
        for (int e = 0; e < E; ++e) {
            const int *en = &h.elem[9 * e];
            double *c = &h.qc[8 * e];
            c[0] = h.X[2 * en[0]];
            c[1] = h.X[2 * en[0] + 1];
            for (int k = 1; k < 4; ++k) {
                c[2 * k] = min_image(h.X[2 * en[k]], c[0], h.L[0]);
                c[2 * k + 1] = min_image(h.X[2 * en[k] + 1], c[1], h.L[1]);
            }
            double a2 = 0.0;
            bool convex = true;
            for (int k = 0; k < 4; ++k) {
                const double *pa = c + 2 * k, *pb = c + 2 * ((k + 1) % 4), *pc = c + 2 * ((k + 2) % 4);
                a2 += pa[0] * pb[1] - pa[1] * pb[0];
                if (!((pb[0] - pa[0]) * (pc[1] - pb[1]) - (pb[1] - pa[1]) * (pc[0] - pb[0]) > 0.0)) convex = false;
            }
            h.area[e] = 0.5 * a2;
            if (!convex) {
                snprintf(buf, sizeof buf, "quadrilateral %d is not strictly convex and counter-clockwise", e);
                why = buf;
                return ALE_LB_EMESH;
            }
            // edge and centre nodes where the bilinear map puts them
            for (int s = 4; s < 9; ++s) {
                double x[2], J[4];
                q2_map_host(c, QXI[s], QETA[s], x, J);
                const int a = en[s];
                const double ex = min_image(h.X[2 * a], x[0], h.L[0]) - x[0];
                const double ey = min_image(h.X[2 * a + 1], x[1], h.L[1]) - x[1];
                if (std::fabs(ex) + std::fabs(ey) > 1e-9 * std::sqrt(std::fabs(h.area[e]))) {
                    snprintf(buf, sizeof buf, "node %d of quadrilateral %d is not at its bilinear position", s, e);
                    why = buf;
                    return ALE_LB_EMESH;
                }
            }
        }
    } else {
        h.ev.resize(6 * size_t(E));
        h.A.resize(4 * size_t(E));
        for (int e = 0; e < E; ++e) {
            const int *en = &h.elem[6 * e];
            double *v = &h.ev[6 * e];
            v[0] = h.X[2 * en[0]];
            v[1] = h.X[2 * en[0] + 1];
            for (int k = 1; k < 3; ++k) {
                v[2 * k] = min_image(h.X[2 * en[k]], v[0], h.L[0]);
                v[2 * k + 1] = min_image(h.X[2 * en[k] + 1], v[1], h.L[1]);
            }
            const double b00 = v[2] - v[0], b01 = v[4] - v[0], b10 = v[3] - v[1], b11 = v[5] - v[1];
            const double det = b00 * b11 - b01 * b10;
            h.area[e] = 0.5 * det;
            if (!(det > 0.0)) {
                snprintf(buf, sizeof buf, "element %d has non-positive area", e);
                why = buf;
                return ALE_LB_EMESH;
            }
            double *A = &h.A[4 * e];
            A[0] = b11 / det;
            A[1] = -b01 / det;
            A[2] = -b10 / det;
            A[3] = b00 / det;
        }
    }
    for (int e = 0; e < E; ++e)
        for (int k = 0; k < NF; ++k) {
            const int n = h.nbr[NF * e + k];
            if (n >= E || n < -2) {
                snprintf(buf, sizeof buf, "neighbour of element %d out of range", e);
                why = buf;
                return ALE_LB_EMESH;
            }
            bool back = false;
            for (int j = 0; n >= 0 && j < NF; ++j) back |= h.nbr[NF * n + j] == e;
            if (n >= 0 && !back) {
                snprintf(buf, sizeof buf, "neighbours of elements %d and %d are not symmetric", e, n);
                why = buf;
                return ALE_LB_EMESH;
            }
            const int c = h.psh[NF * e + k];
            if (c < -4 || c > 4) {
                snprintf(buf, sizeof buf, "periodic shift code of element %d out of range", e);
                why = buf;
                return ALE_LB_EMESH;
            }
        }
    // owner: the containing element of largest area, ties to the lowest caller index
    h.owner.assign(N, -1);
    h.oslot.assign(N, 0);
    for (int e = 0; e < E; ++e)
        for (int k = 0; k < NV; ++k) {
            const int a = h.elem[NV * e + k];
            const int c = h.owner[a];
            if (c < 0 || h.area[e] > h.area[c]) {
                h.owner[a] = e;
                h.oslot[a] = k;
            }
        }
    h.opos.resize(2 * size_t(N));
    for (int a = 0; a < N; ++a) {
        if (h.owner[a] < 0) {
            snprintf(buf, sizeof buf, "node %d belongs to no element", a);
            why = buf;
            return ALE_LB_EMESH;
        }
        node_pos_host(h, h.owner[a], h.oslot[a], &h.opos[2 * a]);
        for (int d = 0; d < 2; ++d)
            if (h.L[d] > 0.0 && std::fabs(h.opos[2 * a + d] - h.X[2 * a + d]) > 1.5 * h.L[d]) {
                snprintf(buf, sizeof buf, "node %d lies more than one period from its owner element", a);
                why = buf;
                return ALE_LB_EMESH;
            }
    }
    // wall nodes, computational into-fluid normals and points B (Sec. IV.A)
    const int NWE = int(h.wedge.size() / 2);
    h.wid.assign(N, -1);
    std::vector<double> nacc(2 * size_t(N), 0.0);
    h.nw = 0;
    for (int w = 0; w < NWE; ++w) {
        const int e = h.wedge[2 * w], k = h.wedge[2 * w + 1];
        if (e < 0 || e >= E || k < 0 || k >= NF || h.nbr[NF * e + k] != -1) {
            snprintf(buf, sizeof buf, "wall edge %d is not a wall-tagged element edge", w);
            why = buf;
            return ALE_LB_EMESH;
        }
        int sl[3];
        edge_slots_host(h, k, sl);
        double pa[2], pb[2];
        node_pos_host(h, e, sl[0], pa);
        node_pos_host(h, e, sl[2], pb);
        const double dx = pb[0] - pa[0], dy = pb[1] - pa[1];
        const double L = std::sqrt(dx * dx + dy * dy);
        const int nodes[3] = {h.elem[NV * e + sl[0]], h.elem[NV * e + sl[2]], h.elem[NV * e + sl[1]]};
        for (int a : nodes) {
            if (h.wid[a] < 0) h.wid[a] = h.nw++;
            nacc[2 * a] += -dy / L;
            nacc[2 * a + 1] += dx / L;
        }
    }
    h.bel.assign(std::max(h.nw, 1), 0);
    h.blam.assign(3 * size_t(std::max(h.nw, 1)), 0.0);
    for (int a = 0; a < N; ++a) {
        const int w = h.wid[a];
        if (w < 0) continue;
        const double L = std::sqrt(nacc[2 * a] * nacc[2 * a] + nacc[2 * a + 1] * nacc[2 * a + 1]);
        double B[2] = {h.opos[2 * a] + dt * (nacc[2 * a] / L), h.opos[2 * a + 1] + dt * (nacc[2 * a + 1] / L)};
        double l[3];
        const int eb = host_walk(h, h.owner[a], B, l);
        if (eb < 0) {
            snprintf(buf, sizeof buf, "point B of wall node %d lies outside the mesh", a);
            why = buf;
            return ALE_LB_EMESH;
        }
        h.bel[w] = eb;
        h.blam[3 * w] = l[0];
        h.blam[3 * w + 1] = l[1];
        h.blam[3 * w + 2] = l[2];
    }
    // Hilbert order of nodes (canonical coordinates) and elements (frame centroids, wrapped)
    h.perm = hilbert_order(h.X);
    h.iperm.assign(N, 0);
    for (int k = 0; k < N; ++k) h.iperm[h.perm[k]] = k;
    std::vector<double> cen(2 * size_t(E));
    const int nc = h.kind == ELEM_Q2 ? 4 : 3;
    for (int e = 0; e < E; ++e) {
        const double *v = h.kind == ELEM_Q2 ? &h.qc[8 * e] : &h.ev[6 * e];
        for (int d = 0; d < 2; ++d) {
            double c = 0.0;
            for (int k = 0; k < nc; ++k) c += v[2 * k + d];
            c /= nc;
            if (h.L[d] > 0.0) c = c - h.L[d] * std::floor(c / h.L[d]);
            cen[2 * e + d] = c;
        }
    }
    h.eperm = hilbert_order(cen);
    h.eiperm.assign(E, 0);
    for (int k = 0; k < E; ++k) h.eiperm[h.eperm[k]] = k;
    return ALE_LB_OK;
}

struct DeviceBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

}  // namespace

int alelb::report_error(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

struct ale_lb {
    std::vector<ale_lb_params_t> prm;
    ale_lb_lattice_t lat{};
    int ncases = 1, motion = 0, flags = 0, check_every = 0;
    int kind = ELEM_P2;      // element kind of every case
    int N = 0, Ncaller = 0, E = 0, NW = 0, NWE = 0;
    std::vector<int> perm;   // node slot -> caller node (-1 = padding)
    std::vector<int> iperm;  // caller node -> node slot
    std::vector<int> case_caller_off;
    hipStream_t st = nullptr;
    bool own_stream = false;
    int device = 0;  // current device at create: the handle's buffers and stream live there
    bool fp32 = false;
    std::vector<DeviceBuf> bufs;
    size_t dev_bytes = 0;
    DevMesh dm{};
    DevState<float> sf{};
    DevState<double> sd{};
    CaseStatic *d_cs = nullptr;
    CaseClock *d_cc = nullptr;
    double *d_tcase = nullptr;
    int cur = 0;
    std::vector<double> t;   // host mirror of each case's time
    int64_t step = 0;
    int *d_err = nullptr;
    double *d_part = nullptr;
    double *d_fout = nullptr;
    int2 *d_case_blocks = nullptr;
    int force_blocks = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int graph_cur = -1;
    // ALE_LB_F_PIPELINE: cases [0, split_case) on st, [split_case, ncases) on st2 (split_case 0: off)
    int split_case = 0, split_node = 0;
    hipStream_t st2 = nullptr;
    hipEvent_t ev_a = nullptr, ev_b = nullptr;
    // launch schedule and the tables of the tile kernel
    Schedule sch{0, 1, 256, 1};
    TileArgs ta{};
    void *tile_buf[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    int tile_overflow = 0;             // tiles on the global path
    int tile_rings = 0, tile_limit = -1;  // what the tables were built for
    int lds_limit = 0;                 // cap on a tile workgroup's LDS (0: the device's)
    std::vector<ElemRec> hel;          // element records (host copy, for the tile tables)
    std::vector<int> inc_off, inc;     // node slot -> elements holding it (CSR)
    // the batch of steps in flight starts here (restoring the last good step after a failure)
    std::vector<double> t_mark;
    int64_t step_mark = 0;

    // the caller's allocator (ale_lb_params_t::dev_alloc / dev_free), else hipMalloc / hipFree
    void *(*dalloc)(size_t, void *) = nullptr;
    void (*dfree)(void *, void *) = nullptr;
    void *actx = nullptr;
    hipError_t dmalloc(void **p, size_t bytes)
    {
        if (!dalloc) return hipMalloc(p, bytes);
        *p = dalloc(bytes, actx);
        if (!*p) return hipErrorOutOfMemory;
        if (reinterpret_cast<uintptr_t>(*p) & 255) {
            dfree(*p, actx);
            *p = nullptr;
            return hipErrorInvalidValue;
        }
        return hipSuccess;
    }
    void dmfree(void *p)
    {
        if (!p) return;
        if (dfree)
            dfree(p, actx);
        else
            (void)hipFree(p);
    }
    void *alloc(size_t bytes, int *status)
    {
        void *p = nullptr;
        if (*status) return nullptr;  // an earlier allocation of the same set-up failed
        if (bytes == 0) bytes = 8;
        hipError_t e = dmalloc(&p, bytes);
        if (e != hipSuccess) {
            *status = fail(e == hipErrorOutOfMemory ? ALE_LB_ENOMEM
                           : e == hipErrorInvalidValue ? ALE_LB_EINVAL : ALE_LB_EDEVICE,
                           "device allocation of %zu bytes: %s", bytes,
                           e == hipErrorInvalidValue ? "not 256-byte aligned" : hipGetErrorString(e));
            return nullptr;
        }
        bufs.push_back({p, bytes});
        dev_bytes += bytes;
        return p;
    }
    template <typename T>
    T *upload(const std::vector<T> &v, int *status)
    {
        T *p = static_cast<T *>(alloc(sizeof(T) * v.size(), status));
        if (!p) return nullptr;
        if (!v.empty()) {
            hipError_t e = hipMemcpy(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice);
            if (e != hipSuccess) {
                *status = fail(ALE_LB_EDEVICE, "upload: %s", hipGetErrorString(e));
                return nullptr;
            }
        }
        return p;
    }
    void drop_graph()
    {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        gexec = nullptr;
        graph = nullptr;
        graph_cur = -1;
    }
    void free_tiles()
    {
        for (auto &b : tile_buf) {
            dmfree(b);
            b = nullptr;
        }
        ta = TileArgs{};
        tile_overflow = 0;
        tile_rings = 0;
        tile_limit = -1;
    }
    const TileArgs *tiles() const { return tiled(sch) ? &ta : nullptr; }
    ~ale_lb()
    {
        free_tiles();
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        if (st2) (void)hipStreamSynchronize(st2);
        for (auto &b : bufs) dmfree(b.p);
        if (ev_a) (void)hipEventDestroy(ev_a);
        if (ev_b) (void)hipEventDestroy(ev_b);
        if (st2) (void)hipStreamDestroy(st2);
        if (own_stream) (void)hipStreamDestroy(st);
    }
};

namespace {

template <typename R>
int alloc_state(ale_lb *h, DevState<R> &s)
{
    int st = ALE_LB_OK;
    const size_t N = h->N;
    for (int b = 0; b < 2; ++b) {
        s.pop[b] = static_cast<R *>(h->alloc(sizeof(R) * NPOP * N, &st));
        s.mac[b] = static_cast<R *>(h->alloc(sizeof(R) * 4 * N, &st));
        if (st) return st;
        HIP_OK(hipMemset(s.pop[b], 0, sizeof(R) * NPOP * N));
        HIP_OK(hipMemset(s.mac[b], 0, sizeof(R) * 4 * N));
    }
    s.ft = static_cast<R *>(h->alloc(sizeof(R) * NPOP * N, &st));
    s.W = static_cast<R *>(h->alloc(sizeof(R) * 2 * N, &st));
    s.Xc = static_cast<R *>(h->alloc(sizeof(R) * 2 * N, &st));
    s.Xs[0] = static_cast<R *>(h->alloc(sizeof(R) * 2 * N, &st));
    s.Xs[1] = static_cast<R *>(h->alloc(sizeof(R) * 2 * N, &st));
    if (st) return st;
    HIP_OK(hipMemset(s.ft, 0, sizeof(R) * NPOP * N));
    HIP_OK(hipMemset(s.W, 0, sizeof(R) * 2 * N));
    HIP_OK(hipMemset(s.Xc, 0, sizeof(R) * 2 * N));
    HIP_OK(hipMemset(s.Xs[0], 0, sizeof(R) * 2 * N));
    HIP_OK(hipMemset(s.Xs[1], 0, sizeof(R) * 2 * N));
    s.mask = nullptr;
    if (h->flags & ALE_LB_F_KEEP_MASKS) {
        s.mask = static_cast<int *>(h->alloc(sizeof(int) * N, &st));
        if (st) return st;
        HIP_OK(hipMemset(s.mask, 0, sizeof(int) * N));
    }
    s.hint = static_cast<int *>(h->alloc(sizeof(int) * Q * N, &st));
    s.wlist = static_cast<int2 *>(h->alloc(sizeof(int2) * N, &st));
    s.wcount = static_cast<int *>(h->alloc(2 * sizeof(int), &st));  // one counter per half of a split batch
    if (st) return st;
    HIP_OK(hipMemset(s.wcount, 0, 2 * sizeof(int)));
    s.err = h->d_err;
    return ALE_LB_OK;
}

// the clock a step with input buffers `cur` reads (its successor's is the other)
CaseClock *clock_of(ale_lb *h, int cur) { return h->d_cc + size_t(h->ncases) * cur; }

int upload_clock(ale_lb *h);

// both correction-field buffers of the tile state cleared (a new state holds f* itself)
hipError_t clear_x(ale_lb *h)
{
    const size_t b = (h->fp32 ? sizeof(float) : sizeof(double)) * 2 * size_t(h->N);
    for (int k = 0; k < 2; ++k) {
        void *p = h->fp32 ? static_cast<void *>(h->sf.Xs[k]) : static_cast<void *>(h->sd.Xs[k]);
        const hipError_t e = hipMemsetAsync(p, 0, b, h->st);
        if (e != hipSuccess) return e;
    }
    return hipStreamSynchronize(h->st);
}

// The batch of steps about to be enqueued starts from the handle's state.
void mark_batch(ale_lb *h)
{
    h->t_mark = h->t;
    h->step_mark = h->step;
}

// After the work enqueued so far: if a step failed, report it and put the
// handle back at its last good step.  The failing step alone raised error
// bits, with the parity of its input buffers; every kernel of the steps after
// it returned without writing, so those buffers still hold the last good
// state, and that parity's clock holds the failing step's count.  The host
// clock is rebuilt by the same additions the device made since the batch
// began.
int check_err(ale_lb *h)
{
    int err = 0;
    HIP_OK(hipMemcpyAsync(&err, h->d_err, sizeof(int), hipMemcpyDeviceToHost, h->st));
    HIP_OK(hipStreamSynchronize(h->st));
    if (!err) return ALE_LB_OK;
    const int par = (err >> ERR_PARITY) & 3;
    if (par == 1 || par == 2) {
        const int p = par == 1 ? 0 : 1;
        CaseClock ck;
        HIP_OK(hipMemcpy(&ck, clock_of(h, p), sizeof ck, hipMemcpyDeviceToHost));
        const int64_t good = ck.step - 1;
        for (int c = 0; c < h->ncases; ++c) {
            double t = c < int(h->t_mark.size()) ? h->t_mark[c] : h->t[c];
            for (int64_t k = h->step_mark; k < good; ++k) t += h->prm[c].dt;
            h->t[c] = t;
        }
        h->cur = p;
        h->step = good;
    }
    const int zero[2] = {0, 0};
    HIP_OK(hipMemcpyAsync(h->d_err, zero, sizeof(int), hipMemcpyHostToDevice, h->st));
    int *wc = h->fp32 ? h->sf.wcount : h->sd.wcount;
    HIP_OK(hipMemcpyAsync(wc, zero, 2 * sizeof(int), hipMemcpyHostToDevice, h->st));
    const int st = upload_clock(h);  // also drains the stream
    if (st) return st;
    const long long bad = (long long)h->step + 1, last = (long long)h->step;
    if (err & ERR_JAC)
        return fail(ALE_LB_EJAC, "mapping Jacobian det <= 0 in step %lld; the state is that of step %lld", bad, last);
    if (err & ERR_LOCATE)
        return fail(ALE_LB_ELOCATE, "element walk exceeded %d steps in step %lld; the state is that of step %lld",
                    WALK_CAP, bad, last);
    return fail(ALE_LB_ENONFINITE, "non-finite populations in step %lld; the state is that of step %lld", bad, last);
}

template <typename R>
StepArgs<R> step_args(ale_lb *h, DevState<R> &s, int cur)
{
    StepArgs<R> a;
    a.m = h->dm;
    a.s = s;
    a.cur = cur;
    a.clock_next = clock_of(h, cur ^ 1);
    a.flags = h->flags;
    a.node0 = 0;
    a.node1 = h->N;
    a.c0 = 0;
    a.c1 = h->ncases;
    return a;
}

// one half of a split batch: its node slots, cases, wall list and counter
template <typename R>
StepArgs<R> half_args(ale_lb *h, DevState<R> &s, int cur, int half)
{
    StepArgs<R> a = step_args(h, s, cur);
    a.node0 = half ? h->split_node : 0;
    a.node1 = half ? h->N : h->split_node;
    a.c0 = half ? h->split_case : 0;
    a.c1 = half ? h->ncases : h->split_case;
    a.s.wlist = s.wlist + a.node0;
    a.s.wcount = s.wcount + half;
    return a;
}

// the second stream's work so far completes before anything later on the first
int pipe_join(ale_lb *h)
{
    HIP_OK(hipEventRecord(h->ev_b, h->st2));
    HIP_OK(hipStreamWaitEvent(h->st, h->ev_b, 0));
    return ALE_LB_OK;
}

void advance_host_clock(ale_lb *h)
{
    for (int c = 0; c < h->ncases; ++c) h->t[c] = h->t[c] + h->prm[c].dt;
    h->cur ^= 1;
    h->step += 1;
}

// capture two steps (cur, then 1 - cur) as one HIP graph
template <typename R>
int capture_graph(ale_lb *h, DevState<R> &s)
{
    h->drop_graph();
    HIP_OK(hipStreamBeginCapture(h->st, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < 2; ++k) {
        const hipError_t e = launch_step<R>(step_args(h, s, h->cur ^ k), h->d_cs, clock_of(h, h->cur ^ k), h->motion,
                                            h->sch, h->tiles(), h->st, nullptr);
        if (e != hipSuccess) {
            hipGraph_t g;
            (void)hipStreamEndCapture(h->st, &g);
            return fail(ALE_LB_EDEVICE, "graph capture: %s", hipGetErrorString(e));
        }
    }
    HIP_OK(hipStreamEndCapture(h->st, &h->graph));
    HIP_OK(hipGraphInstantiate(&h->gexec, h->graph, nullptr, nullptr, 0));
    h->graph_cur = h->cur;
    return ALE_LB_OK;
}

// Steps of a split batch on two streams: half A (first stream) streams,
// then half B (second stream) streams while A runs its node kernels.  The
// halves share no node, element or case.  A's next streaming waits for B's
// last kernel of the step, so that no kernel of a step starts before every
// error of the step before is visible, which the recovery after a failed step
// needs; two streaming kernels never run at once.
template <typename R>
int do_steps_split(ale_lb *h, DevState<R> &s, int n)
{
    int next_check = h->check_every;
    const TileArgs *ta = h->tiles();
    mark_batch(h);
    for (int k = 0; k < n;) {
        const StepArgs<R> aA = half_args(h, s, h->cur, 0), aB = half_args(h, s, h->cur, 1);
        CaseClock *cc = clock_of(h, h->cur);
        if (k > 0) HIP_OK(hipStreamWaitEvent(h->st, h->ev_b, 0));
        HIP_OK(launch_stream_phase<R>(aA, h->d_cs, cc, h->motion, h->sch, ta, h->st));
        HIP_OK(hipEventRecord(h->ev_a, h->st));
        HIP_OK(hipStreamWaitEvent(h->st2, h->ev_a, 0));
        HIP_OK(launch_stream_phase<R>(aB, h->d_cs, cc, h->motion, h->sch, ta, h->st2));
        HIP_OK(launch_wall_phase<R>(aA, h->d_cs, cc, h->motion, h->sch, h->st));
        HIP_OK(launch_grad_phase<R>(aA, h->d_cs, cc, h->motion, h->sch, h->st));
        HIP_OK(launch_wall_phase<R>(aB, h->d_cs, cc, h->motion, h->sch, h->st2));
        HIP_OK(launch_grad_phase<R>(aB, h->d_cs, cc, h->motion, h->sch, h->st2));
        HIP_OK(hipEventRecord(h->ev_b, h->st2));
        advance_host_clock(h);
        ++k;
        if (h->check_every > 0 && k >= next_check && k < n) {
            int st = pipe_join(h);
            if (!st) st = check_err(h);
            if (st) return st;
            next_check = k + h->check_every;
            mark_batch(h);
        }
    }
    const int st = pipe_join(h);
    return st ? st : check_err(h);
}

template <typename R>
int do_steps(ale_lb *h, DevState<R> &s, int n, hipEvent_t *ev, double *ms)
{
    if (h->split_case > 0 && !ev) return do_steps_split(h, s, n);
    const bool graph = (h->flags & ALE_LB_F_GRAPH) && !ev;
    int k = 0, next_check = h->check_every;
    mark_batch(h);
    while (k < n) {
        if (graph && n - k >= 2) {
            if (!h->gexec || h->graph_cur != h->cur) {
                if (h->gexec && h->graph_cur != h->cur) {
                    // parity differs from the captured pair: one plain step first
                    HIP_OK(launch_step<R>(step_args(h, s, h->cur), h->d_cs, clock_of(h, h->cur), h->motion, h->sch,
                                          h->tiles(), h->st, nullptr));
                    advance_host_clock(h);
                    ++k;
                    continue;
                }
                const int st = capture_graph(h, s);
                if (st) return st;
            }
            HIP_OK(hipGraphLaunch(h->gexec, h->st));
            advance_host_clock(h);
            advance_host_clock(h);
            k += 2;
        } else {
            HIP_OK(launch_step<R>(step_args(h, s, h->cur), h->d_cs, clock_of(h, h->cur), h->motion, h->sch,
                                  h->tiles(), h->st, ev));
            if (ev) {
                HIP_OK(hipEventSynchronize(ev[NKERNELS]));
                float d;
                for (int q = 0; q < NKERNELS; ++q) {
                    HIP_OK(hipEventElapsedTime(&d, ev[q], ev[q + 1]));
                    ms[q] += d;
                }
                HIP_OK(hipEventElapsedTime(&d, ev[0], ev[NKERNELS]));
                ms[NKERNELS] += d;
            }
            advance_host_clock(h);
            ++k;
        }
        if (h->check_every > 0 && k >= next_check && k < n) {
            const int st = check_err(h);
            if (st) return st;
            next_check = k + h->check_every;
            mark_batch(h);
        }
    }
    return check_err(h);
}

// ---- tables of the tile kernel ----
// LDS a tile workgroup may use: the device's per-workgroup limit (at most
// PATCH_LDS_LIMIT) less the kernel's static LDS; and the part of it a patch
// may take, which the handle's cap can lower
int tile_budget(ale_lb *h, size_t *device, size_t *patch)
{
    int dev = 0, maxlds = 0;
    HIP_OK(hipGetDevice(&dev));
    HIP_OK(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    *device = std::min<size_t>(size_t(maxlds), PATCH_LDS_LIMIT) - 64;  // the abort flag and alignment
    *patch = h->lds_limit > 0 ? std::min<size_t>(*device, size_t(h->lds_limit)) : *device;
    return ALE_LB_OK;
}

// Where the walk of direction i at node slot v starts: the element holding v
// that contains a point just upwind of it along -c_i (the departure point of
// a mesh at rest, for a displacement below the element's size), else the
// owner (the rest direction, and directions that leave the domain at v).
// Inside the domain the element a walk ends in does not depend on where it
// starts (up to a point on a shared edge), and a nearby start saves walk
// steps.  Next to a boundary the visibility walk can end at a wall or the far
// field from one start and not from another (a non-convex boundary such as
// the trailing edge), and the reading takes the walk from the owner: nodes
// whose elements touch a boundary edge start every walk there, and the
// kernel walks again from the owner whenever a walk from elsewhere ends at
// the boundary.
int walk_start(const ale_lb *h, int v, int i, int owner)
{
    static const int cx[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1}, cy[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    if (i == 0) return owner;
    for (int j = h->inc_off[v]; j < h->inc_off[v + 1]; ++j) {
        const int4 nb = h->hel[h->inc[j]].nb;
        if (nb.x < 0 || nb.y < 0 || nb.z < 0) return owner;
    }
    const double cn = std::sqrt(double(cx[i] * cx[i] + cy[i] * cy[i]));
    int best = owner;
    double best_min = -1e300;
    for (int j = h->inc_off[v]; j < h->inc_off[v + 1]; ++j) {
        const int e = h->inc[j];
        const ElemRec &r = h->hel[e];
        const double det = r.a01.x * r.a23.y - r.a01.y * r.a23.x;  // of the map (x - v0) -> (l1, l2)
        if (!(det != 0.0)) continue;
        // vertices from the inverse map: v1 - v0 = (A3, -A2) / det, v2 - v0 = (-A1, A0) / det
        const double e1x = r.a23.y / det, e1y = -r.a23.x / det, e2x = -r.a01.y / det, e2y = r.a01.x / det;
        int s2 = 0;
        while (s2 < 6 && r.n[s2] != v) ++s2;
        if (s2 == 6) continue;
        // the node's barycentrics in e, then its position relative to v0
        double lam[3] = {0, 0, 0};
        if (s2 < 3) {
            lam[s2] = 1.0;
        } else {
            lam[(s2 - 2) % 3] = 0.5;
            lam[(s2 - 1) % 3] = 0.5;
        }
        const double px = lam[1] * e1x + lam[2] * e2x, py = lam[1] * e1y + lam[2] * e2y;
        const double d = 1e-3 * std::sqrt(std::fabs(e1x * e2y - e1y * e2x));
        const double qx = px - d * cx[i] / cn, qy = py - d * cy[i] / cn;
        const double l1 = r.a01.x * qx + r.a01.y * qy, l2 = r.a23.x * qx + r.a23.y * qy;
        const double mn = std::min(std::min(l1, l2), 1.0 - l1 - l2);
        if (mn > best_min) {
            best_min = mn;
            best = e;
        }
    }
    return best_min >= -1e-12 ? best : owner;
}

// Patches of tiles of T node slots: every element holding a node of the tile
// (and their neighbours for rings = 2), every node of those elements, the
// tile's own slots first; element records with local node and neighbour
// indices.  Tiles whose patch exceeds the LDS budget are marked for the
// global path (the workgroup still holds its T output rows in LDS).
int build_tiles(ale_lb *h, int T, int rings)
{
    const int N = h->N, E = h->E;
    if (N % T) return fail(ALE_LB_EINVAL, "tile of %d nodes does not divide the node slots", T);
    size_t budget = 0, dev_budget = 0;
    int st = tile_budget(h, &dev_budget, &budget);
    if (st) return st;
    const int pop_bytes = h->fp32 ? 4 : 8;
    if (tile_lds_bytes(0, T, pop_bytes, T) > dev_budget)
        return fail(ALE_LB_EUNSUPPORTED, "no LDS left for tiles of %d nodes (%zu bytes per workgroup)", T,
                    dev_budget);
    if (h->inc_off.empty()) {
        // node slot -> elements holding it
        h->inc_off.assign(N + 1, 0);
        for (int e = 0; e < E; ++e)
            for (int s2 = 0; s2 < 6; ++s2) h->inc_off[h->hel[e].n[s2] + 1]++;
        for (int v = 0; v < N; ++v) h->inc_off[v + 1] += h->inc_off[v];
        h->inc.assign(h->inc_off[N], 0);
        std::vector<int> fill(h->inc_off.begin(), h->inc_off.end() - 1);
        for (int e = 0; e < E; ++e)
            for (int s2 = 0; s2 < 6; ++s2) h->inc[fill[h->hel[e].n[s2]]++] = e;
    }
    std::vector<int> own(N);
    HIP_OK(hipMemcpy(own.data(), h->dm.own, sizeof(int) * N, hipMemcpyDeviceToHost));
    const int tiles = N / T;
    std::vector<int4> hdr(tiles);
    std::vector<uint4> rec;
    std::vector<int> pelem, pnode, es, ns;
    std::vector<uint4> start(N, make_uint4(0, 0, 0, 0));
    std::vector<int> mark_e(E, -1), loc_e(E, 0), mark_n(N, -1), loc_n(N, 0);
    rec.reserve(size_t(N) * 3);
    pelem.reserve(size_t(N));
    pnode.reserve(size_t(N) * 2);
    for (int t = 0; t < tiles; ++t) {
        es.clear();
        ns.clear();
        for (int v = t * T; v < (t + 1) * T; ++v) {
            if (h->perm[v] < 0) continue;
            for (int j = h->inc_off[v]; j < h->inc_off[v + 1]; ++j) {
                const int e = h->inc[j];
                if (mark_e[e] != t) {
                    mark_e[e] = t;
                    es.push_back(e);
                }
            }
        }
        for (int r = 1; r < rings; ++r) {
            const size_t n0 = es.size();
            for (size_t j = 0; j < n0; ++j) {
                const int4 nb = h->hel[es[j]].nb;
                for (int g : {nb.x, nb.y, nb.z})
                    if (g >= 0 && mark_e[g] != t) {
                        mark_e[g] = t;
                        es.push_back(g);
                    }
            }
        }
        std::sort(es.begin(), es.end());
        for (size_t q = 0; q < es.size(); ++q) loc_e[es[q]] = int(q);
        // the tile's own slots first, in order, then the other patch nodes ascending
        for (int v = t * T; v < (t + 1) * T; ++v) {
            mark_n[v] = t;
            loc_n[v] = v - t * T;
        }
        for (int e : es)
            for (int s2 = 0; s2 < 6; ++s2) {
                const int v = h->hel[e].n[s2];
                if (mark_n[v] != t) {
                    mark_n[v] = t;
                    ns.push_back(v);
                }
            }
        std::sort(ns.begin(), ns.end());
        for (size_t q = 0; q < ns.size(); ++q) loc_n[ns[q]] = T + int(q);
        const int npe = int(es.size()), npn = T + int(ns.size());
        if (npe > TILE_MAX_LOCAL - 1 || npn > TILE_MAX_LOCAL)
            return fail(ALE_LB_EUNSUPPORTED, "tile %d: patch of %d elements / %d nodes exceeds %d", t, npe, npn,
                        TILE_MAX_LOCAL);
        hdr[t] = make_int4(int(pelem.size()), npe, int(pnode.size()), npn);
        for (int e : es) {
            const ElemRec &r = h->hel[e];
            uint4 w[4];
            std::memcpy(&w[0], &r.v0, 16);
            std::memcpy(&w[1], &r.a01, 16);
            std::memcpy(&w[2], &r.a23, 16);
            unsigned ln[6], lb[3];
            for (int s2 = 0; s2 < 6; ++s2) ln[s2] = unsigned(loc_n[r.n[s2]]);
            const int nb[3] = {r.nb.x, r.nb.y, r.nb.z};
            for (int k = 0; k < 3; ++k)
                lb[k] = nb[k] == -1 ? TL_WALL : nb[k] < 0 ? TL_FAR : mark_e[nb[k]] == t ? unsigned(loc_e[nb[k]]) : TL_OUT;
            w[3].x = ln[0] | ln[1] << 10 | ln[2] << 20;
            w[3].y = ln[3] | ln[4] << 10 | ln[5] << 20;
            w[3].z = lb[0] | lb[1] << 10 | lb[2] << 20;
            w[3].w = unsigned(r.nb.w);  // shift codes + 4, 4 bits per edge
            rec.insert(rec.end(), w, w + 4);
            pelem.push_back(e);
        }
        for (int v = t * T; v < (t + 1) * T; ++v) {
            pnode.push_back(v);
            if (h->perm[v] < 0) continue;
            unsigned w[3] = {0, 0, 0};
            for (int i = 0; i < Q; ++i) {
                const int e = walk_start(h, v, i, own[v]);
                w[i / 3] |= unsigned(loc_e[e]) << (10 * (i % 3));
            }
            start[v] = make_uint4(w[0], w[1], w[2], unsigned(loc_e[own[v]]));
        }
        pnode.insert(pnode.end(), ns.begin(), ns.end());
    }
    // LDS layout size: the largest patch, shrunk until it fits the budget;
    // tiles above the caps take the global path (all of them if not even the
    // output rows fit the patch budget)
    int pe_max = 0, pn_max = T;
    for (const int4 &d : hdr) {
        pe_max = std::max(pe_max, d.y);
        pn_max = std::max(pn_max, d.w);
    }
    if (tile_lds_bytes(0, T, pop_bytes, T) > budget) {
        pe_max = -1;
        pn_max = T;
    }
    while (pe_max >= 0 && tile_lds_bytes(pe_max, pn_max, pop_bytes, T) > budget) {
        pe_max = pe_max * 15 / 16;
        pn_max = std::max(T, pn_max * 15 / 16);
    }
    int overflow = 0;
    for (int4 &d : hdr)
        if (d.y > pe_max || d.w > pn_max) {
            d.y = -1;
            ++overflow;
        }
    h->free_tiles();
    h->drop_graph();
    const void *src[5] = {hdr.data(), rec.data(), pelem.data(), pnode.data(), start.data()};
    const size_t bytes[5] = {sizeof(int4) * hdr.size(), sizeof(uint4) * rec.size(), sizeof(int) * pelem.size(),
                             sizeof(int) * pnode.size(), sizeof(uint4) * start.size()};
    for (int k = 0; k < 5; ++k) {
        void *b = nullptr;
        hipError_t e = h->dmalloc(&b, std::max<size_t>(bytes[k], 16));
        if (e == hipSuccess && bytes[k]) e = hipMemcpy(b, src[k], bytes[k], hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            h->dmfree(b);
            h->free_tiles();
            return fail(e == hipErrorOutOfMemory ? ALE_LB_ENOMEM : ALE_LB_EDEVICE, "tile tables: %s",
                        hipGetErrorString(e));
        }
        h->tile_buf[k] = b;
    }
    h->ta.hdr = static_cast<const int4 *>(h->tile_buf[0]);
    h->ta.rec = static_cast<const uint4 *>(h->tile_buf[1]);
    h->ta.pelem = static_cast<const int *>(h->tile_buf[2]);
    h->ta.pnode = static_cast<const int *>(h->tile_buf[3]);
    h->ta.start = static_cast<const uint4 *>(h->tile_buf[4]);
    h->ta.pe_max = std::max(pe_max, 0);
    h->ta.pn_max = pn_max;
    h->ta.tile = T;
    h->tile_overflow = overflow;
    h->tile_rings = rings;
    h->tile_limit = h->lds_limit;
    return ALE_LB_OK;
}

template <typename R>
int convert_state(ale_lb *h, DevState<R> &s, bool to_tile)
{
    // one-wave -> tile: the stored populations are f* (X = 0); tile -> one-wave: f* = f' + dt A X
    if (to_tile)
        HIP_OK(hipMemsetAsync(s.Xs[h->cur], 0, sizeof(R) * 2 * size_t(h->N), h->st));
    else
        HIP_OK(launch_fold_x<R>(h->dm, s.pop[h->cur], s.Xs[h->cur], h->d_cs, h->st));
    HIP_OK(hipStreamSynchronize(h->st));
    return ALE_LB_OK;
}

int set_schedule(ale_lb *h, const Schedule &sc)
{
    if (sc.node_block != 64 && sc.node_block != 128 && sc.node_block != 256)
        return fail(ALE_LB_EINVAL, "node block must be 64, 128 or 256 (got %d)", sc.node_block);
    if (sc.waves != 0 && sc.waves != 2 && sc.waves != 4)
        return fail(ALE_LB_EINVAL, "streaming schedule takes 0, 2 or 4 waves (got %d)", sc.waves);
    if (h->kind == ELEM_Q2 && sc.waves != 0)
        return fail(ALE_LB_EUNSUPPORTED, "quadrilateral meshes run the one-wave streaming kernel only (waves = 0)");
    const bool tile = tiled(sc);
    if (!tile && sc.groups != 1 && sc.groups != 4 && sc.groups != 8)
        return fail(ALE_LB_EINVAL, "one-wave schedules take 1, 4 or 8 node groups (got %d)", sc.groups);
    if (tile && (sc.groups < 1 || sc.groups > 3))
        return fail(ALE_LB_EINVAL, "tile schedules take 1, 2 or 3 direction groups (got %d)", sc.groups);
    if (tile && sc.rings != 1 && sc.rings != 2) return fail(ALE_LB_EINVAL, "patch radius must be 1 or 2");
    if (tile && (h->ta.tile != 64 * sc.waves || h->tile_rings != sc.rings || h->tile_limit != h->lds_limit)) {
        const int st = build_tiles(h, 64 * sc.waves, sc.rings);
        if (st) return st;
    }
    if (tile != tiled(h->sch)) {
        const int st = h->fp32 ? convert_state(h, h->sf, tile) : convert_state(h, h->sd, tile);
        if (st) return st;
    }
    h->drop_graph();
    h->sch = sc;
    if (!tile) h->sch.rings = 0;
    return ALE_LB_OK;
}

// Mesh-size bucket of the tuning cache: precision, motion law, element kind, number of cases,
// and log2 of the total and of the mean per-case node count.
struct TuneKey {
    int fp32, motion, kind, ncases, lg_total, lg_mean;
    bool operator<(const TuneKey &o) const
    {
        return std::tie(fp32, motion, kind, ncases, lg_total, lg_mean) <
               std::tie(o.fp32, o.motion, o.kind, o.ncases, o.lg_total, o.lg_mean);
    }
};
std::map<TuneKey, Schedule> g_tune_cache;
std::mutex g_tune_mutex;

TuneKey tune_key(const ale_lb *h)
{
    auto lg = [](double v) { return int(std::floor(std::log2(std::max(v, 1.0)))); };
    return TuneKey{h->fp32 ? 1 : 0, h->motion, h->kind, h->ncases, lg(double(h->Ncaller)),
                   lg(double(h->Ncaller) / h->ncases)};
}

// time `reps` launches of a step's streaming kernel and correction passes
// (stream_kernel), or of the correction passes alone, on the current state:
// its inputs are read and the step's outputs written
template <typename R>
int time_launches(ale_lb *h, DevState<R> &s, bool stream_kernel, int reps, double *ms)
{
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    const StepArgs<R> a = step_args(h, s, h->cur);
    hipError_t e = hipSuccess;
    for (int k = 0; k < reps + 1 && e == hipSuccess; ++k) {
        if (k == 1) e = hipEventRecord(e0, h->st);
        if (e == hipSuccess && stream_kernel)
            e = launch_stream_only<R>(a, h->d_cs, clock_of(h, h->cur), h->motion, h->sch, h->tiles(), h->st);
        if (e == hipSuccess)
            e = launch_node_kernels_only<R>(a, h->d_cs, clock_of(h, h->cur), h->motion, h->sch, h->st);
    }
    if (e == hipSuccess) e = hipEventRecord(e1, h->st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float d = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&d, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIP_OK(e);
    *ms = double(d) / reps;
    return ALE_LB_OK;
}

// Grid search over the step's launch schedule: the one-wave streaming kernel
// with 1, 4 or 8 node groups (with k_collide), the tile kernel with 128 or
// 256 nodes per tile, patch radius 1 or 2 and 1, 2 or 3 direction groups
// (with k_grad2), each timed as streaming kernel + correction passes; then
// the node kernels' block size.
// Timed on the handle's current state: the step's outputs are rewritten by
// the timing launches, its inputs (current populations, moments, correction
// field, clock) are left as they were.
template <typename R>
int autotune(ale_lb *h, DevState<R> &s, int reps, double *best_ms)
{
    // both clock buffers: the timed node kernels write the next step's
    std::vector<CaseClock> saved(2 * size_t(h->ncases));
    HIP_OK(hipMemcpyAsync(saved.data(), h->d_cc, sizeof(CaseClock) * saved.size(), hipMemcpyDeviceToHost, h->st));
    const Schedule cand[] = {{0, 0, 256, 1}, {0, 0, 256, 4}, {0, 0, 256, 8}, {2, 1, 256, 1}, {2, 1, 256, 2},
                             {2, 1, 256, 3}, {2, 2, 256, 2}, {4, 1, 256, 1}, {4, 1, 256, 2}, {4, 1, 256, 3}};
    Schedule best = h->sch;
    double tbest = 1e300;
    int st = ALE_LB_OK;
    mark_batch(h);
    for (const Schedule &c : cand) {
        if (h->kind == ELEM_Q2 && c.waves != 0) continue;
        st = set_schedule(h, c);
        if (st == ALE_LB_EUNSUPPORTED) {
            st = ALE_LB_OK;
            continue;  // no room for this tile size
        }
        if (st) break;
        double ms = 0.0;
        if ((st = time_launches(h, s, true, reps, &ms))) break;
        if (ms < tbest) {
            tbest = ms;
            best = c;
        }
    }
    if (!st) st = set_schedule(h, best);
    double tnode = 1e300;
    int best_nb = 256;
    for (int nb : {64, 128, 256}) {
        if (st) break;
        h->sch.node_block = nb;
        double ms = 0.0;
        if ((st = time_launches(h, s, false, reps, &ms))) break;
        if (ms < tnode) {
            tnode = ms;
            best_nb = nb;
        }
    }
    h->sch.node_block = best_nb;
    hipError_t e = hipMemcpyAsync(h->d_cc, saved.data(), sizeof(CaseClock) * saved.size(), hipMemcpyHostToDevice, h->st);
    if (e == hipSuccess) e = hipMemsetAsync(s.wcount, 0, 2 * sizeof(int), h->st);
    if (e == hipSuccess) e = hipStreamSynchronize(h->st);
    if (!st && e != hipSuccess) st = fail(ALE_LB_EDEVICE, "autotune: %s", hipGetErrorString(e));
    if (!st) st = check_err(h);
    if (best_ms) *best_ms = tbest;
    return st;
}

// device [slots][C] -> host [C][caller nodes].  Populations (pops) are stored
// as deviations from their case's reference and come out whole; with X (a
// tile schedule's state) they are the post-collision populations
// f'_i + dt A_ia X_a.
template <typename R>
int fetch_nodes(ale_lb *h, const R *src, int C, double *out, bool pops = false, const R *X = nullptr)
{
    const size_t N = h->N, M = h->Ncaller;
    double *d = nullptr;
    HIP_OK(h->dmalloc(reinterpret_cast<void **>(&d), sizeof(double) * C * N));
    std::vector<double> tmp(size_t(C) * N);
    hipError_t e = launch_convert<R>(src, d, N, C, h->st, pops ? &h->dm : nullptr, pops ? h->d_cs : nullptr, X);
    if (e == hipSuccess) e = hipMemcpyAsync(tmp.data(), d, sizeof(double) * C * N, hipMemcpyDeviceToHost, h->st);
    if (e == hipSuccess) e = hipStreamSynchronize(h->st);
    h->dmfree(d);
    HIP_OK(e);
    for (size_t c = 0; c < size_t(C); ++c)
        for (size_t k = 0; k < N; ++k)
            if (h->perm[k] >= 0) out[c * M + h->perm[k]] = tmp[c * N + k];
    return ALE_LB_OK;
}

// host [C][caller nodes] -> device [slots][C] (padding slots keep harmless
// values); populations (pops) are stored as deviations from the reference
template <typename R>
int put_nodes(ale_lb *h, const double *in, int C, R *dst, bool pops = false)
{
    const size_t N = h->N, M = h->Ncaller;
    std::vector<double> tmp(size_t(C) * N, 0.0);
    for (size_t c = 0; c < size_t(C); ++c)
        for (size_t k = 0; k < N; ++k)
            tmp[c * N + k] = h->perm[k] >= 0 ? in[c * M + h->perm[k]] : (c == 0 || c == 3 ? 1.0 : 0.0);
    double *d = nullptr;
    HIP_OK(h->dmalloc(reinterpret_cast<void **>(&d), sizeof(double) * C * N));
    hipError_t e = hipMemcpyAsync(d, tmp.data(), sizeof(double) * C * N, hipMemcpyHostToDevice, h->st);
    if (e == hipSuccess) e = launch_convert_back<R>(d, dst, N, C, h->st, pops ? &h->dm : nullptr, pops ? h->d_cs : nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(h->st);
    h->dmfree(d);
    HIP_OK(e);
    return ALE_LB_OK;
}

// Set the device clock to the host's times: the buffer of the step last
// completed holds t (the forces read it), and the next step's is primed with
// k_clock (t + dt and the motion factors of that step).
int upload_clock(ale_lb *h)
{
    std::vector<CaseClock> cc(2 * size_t(h->ncases));
    for (size_t c = 0; c < cc.size(); ++c) {
        std::memset(&cc[c], 0, sizeof(CaseClock));
        cc[c].t = h->t[c % h->ncases];
        cc[c].step = h->step;
    }
    HIP_OK(hipMemcpyAsync(h->d_cc, cc.data(), sizeof(CaseClock) * cc.size(), hipMemcpyHostToDevice, h->st));
    HIP_OK(launch_clock(h->d_cs, clock_of(h, h->cur), h->ncases, h->st));
    HIP_OK(hipStreamSynchronize(h->st));
    return ALE_LB_OK;
}

int create_impl(const ale_lb_mesh_t *meshes, const ale_lb_lattice_t *lattice, const ale_lb_params_t *params,
                int ncases, ale_lb_t **out)
{
    if (!meshes || !lattice || !params || !out) return fail(ALE_LB_EINVAL, "null argument");
    *out = nullptr;
    if (ncases < 1 || ncases > 255) return fail(ALE_LB_EINVAL, "a batch holds 1 to 255 cases (got %d)", ncases);
    if (lattice->Q != 9) return fail(ALE_LB_EUNSUPPORTED, "only the D2Q9 lattice is supported (Q = %d)", lattice->Q);
    if (lattice->shift[0] != 0.0 || lattice->shift[1] != 0.0)
        return fail(ALE_LB_EUNSUPPORTED, "shifted lattices are not supported");
    if (!(lattice->gamma > 1.0) || !(lattice->Pr > 0.0)) return fail(ALE_LB_EINVAL, "gamma must exceed 1 and Pr be positive");
    for (int c = 0; c < ncases; ++c) {
        const ale_lb_mesh_t *mesh = &meshes[c];
        const ale_lb_params_t *p = &params[c];
        if (mesh->n_nodes <= 0 || mesh->n_elems <= 0 || !mesh->X || !mesh->elem || !mesh->nbr)
            return fail(ALE_LB_EINVAL, "case %d: empty mesh", c);
        if (!(p->dt > 0.0) || !(p->mu >= 0.0)) return fail(ALE_LB_EINVAL, "case %d: dt must be positive, mu non-negative", c);
        if (p->precision != ALE_LB_FP64 && p->precision != ALE_LB_FP32)
            return fail(ALE_LB_EINVAL, "case %d: unknown precision %d", c, p->precision);
        if (p->motion < 0 || p->motion > 3) return fail(ALE_LB_EINVAL, "case %d: unknown motion law %d", c, p->motion);
        if (mesh->n_wall_edges < 0 || (mesh->n_wall_edges > 0 && !mesh->wall_edges))
            return fail(ALE_LB_EINVAL, "case %d: bad wall-edge list", c);
        if (p->precision != params[0].precision || p->motion != params[0].motion || p->flags != params[0].flags ||
            p->stream != params[0].stream)
            return fail(ALE_LB_EINVAL, "case %d: precision, motion law, flags and stream must match case 0", c);
        const int nv = mesh->nodes_per_elem == 0 ? 6 : mesh->nodes_per_elem;
        if (nv != 6 && nv != 9)
            return fail(ALE_LB_EINVAL, "case %d: elements have 6 (P2) or 9 (Q2) nodes, not %d", c, nv);
        const int nv0 = meshes[0].nodes_per_elem == 0 ? 6 : meshes[0].nodes_per_elem;
        if (nv != nv0) return fail(ALE_LB_EINVAL, "case %d: element kind must match case 0", c);
    }
    if (bool(params[0].dev_alloc) != bool(params[0].dev_free))
        return fail(ALE_LB_EINVAL, "dev_alloc and dev_free must be given together");
    ale_lb *h = new ale_lb();
    if (hipGetDevice(&h->device) != hipSuccess) h->device = -1;  // the first allocation reports it
    h->dalloc = params[0].dev_alloc;
    h->dfree = params[0].dev_free;
    h->actx = params[0].alloc_ctx;
    h->prm.assign(params, params + ncases);
    h->lat = *lattice;
    h->ncases = ncases;
    h->motion = params[0].motion;
    h->flags = params[0].flags;
    h->check_every = params[0].check_every;
    h->st = static_cast<hipStream_t>(params[0].stream);
    h->fp32 = params[0].precision == ALE_LB_FP32;
    if ((h->flags & ALE_LB_F_GRAPH) && !h->st) {
        // graph capture needs a stream other than the null stream
        if (hipStreamCreate(&h->st) != hipSuccess) {
            delete h;
            return fail(ALE_LB_EDEVICE, "could not create a stream for graph capture");
        }
        h->own_stream = true;
    }

    std::vector<HostMesh> cm(ncases);
    std::vector<int> node_off(ncases), elem_off(ncases), wn_off(ncases), we_off(ncases);
    h->case_caller_off.assign(ncases, 0);
    for (int c = 0; c < ncases; ++c) {
        const ale_lb_mesh_t *mesh = &meshes[c];
        HostMesh &hm = cm[c];
        hm.N = mesh->n_nodes;
        hm.E = mesh->n_elems;
        hm.kind = mesh->nodes_per_elem == 9 ? ELEM_Q2 : ELEM_P2;
        hm.nv = hm.kind == ELEM_Q2 ? 9 : 6;
        hm.nf = hm.kind == ELEM_Q2 ? 4 : 3;
        hm.X.assign(mesh->X, mesh->X + 2 * size_t(hm.N));
        hm.elem.assign(mesh->elem, mesh->elem + size_t(hm.nv) * hm.E);
        hm.nbr.assign(mesh->nbr, mesh->nbr + size_t(hm.nf) * hm.E);
        hm.psh.assign(size_t(hm.nf) * hm.E, 0);
        if (mesh->pshift) hm.psh.assign(mesh->pshift, mesh->pshift + size_t(hm.nf) * hm.E);
        hm.L[0] = mesh->period[0];
        hm.L[1] = mesh->period[1];
        if (mesh->n_wall_edges > 0) hm.wedge.assign(mesh->wall_edges, mesh->wall_edges + 2 * size_t(mesh->n_wall_edges));
        std::string why;
        const int st = validate_and_derive(hm, params[c].dt, why);
        if (st) {
            delete h;
            if (ncases > 1) return fail(st, "case %d: %s", c, why.c_str());
            return fail(st, "%s", why.c_str());
        }
        node_off[c] = h->N;
        elem_off[c] = h->E;
        wn_off[c] = h->NW;
        we_off[c] = h->NWE;
        h->case_caller_off[c] = h->Ncaller;
        h->N += ((hm.N + CASE_ALIGN - 1) / CASE_ALIGN) * CASE_ALIGN;
        h->Ncaller += hm.N;
        h->E += hm.E;
        h->NW += hm.nw;
        h->NWE += int(hm.wedge.size() / 2);
    }
    const int N = h->N;
    if (h->E >= (1 << 27)) {
        delete h;
        return fail(ALE_LB_EUNSUPPORTED, "at most 2^27 elements per handle (got %d)", h->E);
    }
    // node slots: each case's Hilbert-ordered nodes, then padding up to a multiple of CASE_ALIGN
    std::vector<double2> X(N, make_double2(0.0, 0.0));
    std::vector<int> own(N, 0), widv(N, -1);
    std::vector<uint16_t> oinfo(N, PAD_NODE);
    std::vector<uint8_t> ncase(N, 0);
    h->perm.assign(N, -1);
    h->iperm.assign(h->Ncaller, 0);
    h->kind = cm[0].kind;
    const bool quads = h->kind == ELEM_Q2;
    std::vector<ElemRec> el(quads ? 0 : h->E);
    std::vector<ElemGrad> elg(quads ? 0 : h->E);
    std::vector<ElemRecQ> elq(quads ? h->E : 0);
    std::vector<int> bel(std::max(h->NW, 1), 0);
    std::vector<double> blam(3 * size_t(std::max(h->NW, 1)), 0.0);
    std::vector<int2> wedge(std::max(h->NWE, 1));
    std::vector<double4> wxy(std::max(h->NWE, 1));
    std::vector<int4> fblk;
    std::vector<int2> case_blocks(ncases);
    for (int c = 0; c < ncases; ++c) {
        const HostMesh &hm = cm[c];
        const int slots = ((hm.N + CASE_ALIGN - 1) / CASE_ALIGN) * CASE_ALIGN;
        for (int k = 0; k < slots; ++k) ncase[node_off[c] + k] = uint8_t(c);
        for (int k = 0; k < hm.N; ++k) {
            const int a = hm.perm[k];
            const int slot = node_off[c] + k;
            X[slot] = make_double2(hm.X[2 * a], hm.X[2 * a + 1]);
            own[slot] = elem_off[c] + hm.eiperm[hm.owner[a]];
            int sx = 0, sy = 0;
            if (hm.L[0] > 0.0) sx = int(std::lround((hm.opos[2 * a] - hm.X[2 * a]) / hm.L[0]));
            if (hm.L[1] > 0.0) sy = int(std::lround((hm.opos[2 * a + 1] - hm.X[2 * a + 1]) / hm.L[1]));
            oinfo[slot] = uint16_t(hm.oslot[a] | (((sx + 1) + 3 * (sy + 1)) << 4));
            if (h->motion == ALE_LB_MOTION_PITCH_PLUNGE) {
                // The zone of the blended law that the node and every point of its
                // departure traces lie in.  A trace's midpoint is within dt |c^|/2
                // of the node, |c^| <= sqrt 2 + |v_g|, |v_g| <= |A w| r + |h w| in
                // the rigid zone (0 beyond the blend); the margin d is twice that,
                // and the relative 4e-12 is wider than the kernel's zone tests.
                const double *mp = h->prm[c].motion_p;
                const double rx = hm.X[2 * a] - mp[2], ry = hm.X[2 * a + 1] - mp[3], r2 = rx * rx + ry * ry;
                const double r0 = mp[7], r1 = mp[8];
                const double vmax = std::fabs(mp[0] * mp[1]) * std::fabs(r0) + std::fabs(mp[5] * mp[1]);
                const double d = h->prm[c].dt * (1.5 + vmax);
                const double rin = std::min(r0, r1) - d, rout = r1 + d;
                if (r1 > 0.0 && r2 > rout * rout * (1.0 + 4e-12))
                    oinfo[slot] |= INFO_REST;
                else if (!(r1 > 0.0) || (rin > 0.0 && r2 < rin * rin * (1.0 - 4e-12)))
                    oinfo[slot] |= INFO_RIGID;
            }
            widv[slot] = hm.wid[a] >= 0 ? wn_off[c] + hm.wid[a] : -1;
            h->perm[slot] = h->case_caller_off[c] + a;
            h->iperm[h->case_caller_off[c] + a] = slot;
        }
        for (int k = 0; k < hm.E && quads; ++k) {
            const int e = hm.eperm[k];
            ElemRecQ &r = elq[elem_off[c] + k];
            std::memset(&r, 0, sizeof r);
            for (int q = 0; q < 4; ++q) r.c[q] = make_double2(hm.qc[8 * e + 2 * q], hm.qc[8 * e + 2 * q + 1]);
            for (int s = 0; s < 9; ++s) r.n[s] = node_off[c] + hm.iperm[hm.elem[9 * e + s]];
            int nb[4];
            unsigned codes = 0;
            for (int q = 0; q < 4; ++q) {
                const int n = hm.nbr[4 * e + q];
                nb[q] = n >= 0 ? elem_off[c] + hm.eiperm[n] : n;
                codes |= unsigned(hm.psh[4 * e + q] + 4) << (4 * q);
            }
            r.nb = make_int4(nb[0], nb[1], nb[2], nb[3]);
            r.codes = int(codes);
            r.a2 = 2.0 * hm.area[e];
        }
        for (int k = 0; k < hm.E && !quads; ++k) {
            const int e = hm.eperm[k];
            ElemRec &r = el[elem_off[c] + k];
            r.v0 = make_double2(hm.ev[6 * e], hm.ev[6 * e + 1]);
            r.a01 = make_double2(hm.A[4 * e], hm.A[4 * e + 1]);
            r.a23 = make_double2(hm.A[4 * e + 2], hm.A[4 * e + 3]);
            for (int s = 0; s < 6; ++s) r.n[s] = node_off[c] + hm.iperm[hm.elem[6 * e + s]];
            r.pad[0] = r.pad[1] = 0;
            int nb[3];
            unsigned codes = 0;
            for (int q = 0; q < 3; ++q) {
                const int n = hm.nbr[3 * e + q];
                nb[q] = n >= 0 ? elem_off[c] + hm.eiperm[n] : n;
                codes |= unsigned(hm.psh[3 * e + q] + 4) << (4 * q);
            }
            r.nb = make_int4(nb[0], nb[1], nb[2], int(codes));
            ElemGrad &gr = elg[elem_off[c] + k];
            gr.a01 = r.a01;
            gr.a23 = r.a23;
            for (int s = 0; s < 6; ++s) gr.n[s] = r.n[s];
            gr.pad[0] = gr.pad[1] = 0;
        }
        for (int w = 0; w < hm.nw; ++w) {
            bel[wn_off[c] + w] = elem_off[c] + hm.eiperm[hm.bel[w]];
            for (int q = 0; q < 3; ++q) blam[3 * (wn_off[c] + w) + q] = hm.blam[3 * w + q];
        }
        const int nwe = int(hm.wedge.size() / 2);
        for (int w = 0; w < nwe; ++w) {
            const int e = hm.wedge[2 * w], k = hm.wedge[2 * w + 1];
            wedge[we_off[c] + w] = make_int2(elem_off[c] + hm.eiperm[e], k);
            int sl[3];
            edge_slots_host(hm, k, sl);
            double pa[2], pb[2];
            node_pos_host(hm, e, sl[0], pa);
            node_pos_host(hm, e, sl[2], pb);
            wxy[we_off[c] + w] = make_double4(pa[0], pa[1], pb[0], pb[1]);
        }
        case_blocks[c].x = int(fblk.size());
        for (int b = 0; b < nwe; b += BLOCK)
            fblk.push_back(make_int4(c, we_off[c] + b, we_off[c] + std::min(nwe, b + BLOCK), 0));
        case_blocks[c].y = int(fblk.size());
    }
    h->hel = el;
    h->force_blocks = int(fblk.size());
    if (fblk.empty()) fblk.push_back(make_int4(0, 0, 0, 0));

    int st = ALE_LB_OK;
    DevMesh &dm = h->dm;
    dm.N = N;
    dm.E = h->E;
    dm.NW = h->NW;
    dm.NWE = h->NWE;
    dm.ncases = ncases;
    dm.kind = h->kind;
    dm.X = h->upload(X, &st);
    dm.own = h->upload(own, &st);
    dm.oinfo = h->upload(oinfo, &st);
    dm.ncase = h->upload(ncase, &st);
    dm.wid = h->upload(widv, &st);
    dm.el = quads ? nullptr : h->upload(el, &st);
    dm.elg = quads ? nullptr : h->upload(elg, &st);
    dm.elgf = nullptr;
    dm.Xf = nullptr;
    if (h->fp32 && !quads) {
        // the correction passes of an FP32 state on triangles read these instead
        std::vector<float2> Xf(X.size());
        for (size_t k = 0; k < X.size(); ++k) Xf[k] = make_float2(float(X[k].x), float(X[k].y));
        dm.Xf = h->upload(Xf, &st);
        std::vector<ElemGradF> elgf(elg.size());
        for (size_t e = 0; e < elg.size(); ++e) {
            elgf[e].a01 = make_float2(float(elg[e].a01.x), float(elg[e].a01.y));
            elgf[e].a23 = make_float2(float(elg[e].a23.x), float(elg[e].a23.y));
            for (int q = 0; q < 6; ++q) elgf[e].n[q] = elg[e].n[q];
        }
        dm.elgf = h->upload(elgf, &st);
    }
    dm.elq = quads ? h->upload(elq, &st) : nullptr;
    dm.bel = h->upload(bel, &st);
    dm.blam = h->upload(blam, &st);
    dm.wedge = h->upload(wedge, &st);
    dm.wxy = h->upload(wxy, &st);
    dm.fblk = h->upload(fblk, &st);
    h->d_case_blocks = h->upload(case_blocks, &st);
    h->d_err = static_cast<int *>(h->alloc(sizeof(int), &st));
    h->d_part = static_cast<double *>(h->alloc(sizeof(double) * 6 * std::max(h->force_blocks, 1), &st));
    h->d_fout = static_cast<double *>(h->alloc(sizeof(double) * 6 * ncases, &st));
    h->d_cs = static_cast<CaseStatic *>(h->alloc(sizeof(CaseStatic) * ncases, &st));
    h->d_cc = static_cast<CaseClock *>(h->alloc(sizeof(CaseClock) * 2 * ncases, &st));
    h->d_tcase = static_cast<double *>(h->alloc(sizeof(double) * ncases, &st));
    if (st) {
        delete h;
        return st;
    }
    st = h->fp32 ? alloc_state(h, h->sf) : alloc_state(h, h->sd);
    if (st) {
        delete h;
        return st;
    }
    {
        // every walk starts at the node's owner element, in the owner's frame
        std::vector<int> hint(size_t(Q) * N, 0);
        for (int k = 0; k < N; ++k) {
            if (oinfo[k] & PAD_NODE) continue;
            const int hv = (own[k] << 4) | info_code(oinfo[k]);
            for (int q = 0; q < Q; ++q) hint[size_t(Q) * k + q] = hv;
        }
        int *dh = h->fp32 ? h->sf.hint : h->sd.hint;
        if (hipMemcpy(dh, hint.data(), sizeof(int) * hint.size(), hipMemcpyHostToDevice) != hipSuccess) {
            delete h;
            return fail(ALE_LB_EDEVICE, "hint upload failed");
        }
    }
    std::vector<CaseStatic> cs(ncases);
    for (int c = 0; c < ncases; ++c) {
        const ale_lb_params_t &p = params[c];
        std::memset(&cs[c], 0, sizeof(CaseStatic));
        Phys &ph = cs[c].ph;
        ph.dt = p.dt;
        ph.mu = p.mu;
        ph.gamma = lattice->gamma;
        ph.Pr = lattice->Pr;
        ph.Cv = 1.0 / (lattice->gamma - 1.0);
        ph.Cp = ph.Cv + 1.0;
        ph.iCv = 1.0 / ph.Cv;
        ph.rho_inf = p.rho_inf;
        ph.ux_inf = p.u_inf[0];
        ph.uy_inf = p.u_inf[1];
        ph.T_inf = p.T_inf;
        ph.chord = p.chord;
        ph.refx = p.ref_point[0];
        ph.refy = p.ref_point[1];
        ph.Lx = meshes[c].period[0];
        ph.Ly = meshes[c].period[1];
        cs[c].mo.kind = p.motion;
        for (int k = 0; k < 12; ++k) cs[c].mo.p[k] = p.motion_p[k];
    }
    h->t.resize(ncases);
    for (int c = 0; c < ncases; ++c) h->t[c] = params[c].t0;
    hipError_t e = hipMemcpy(h->d_cs, cs.data(), sizeof(CaseStatic) * ncases, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(h->d_err, 0, sizeof(int));
    if (e == hipSuccess) e = launch_freestream(h->d_cs, ncases, h->st);
    if (e == hipSuccess) e = hipStreamSynchronize(h->st);
    if (e != hipSuccess) {
        delete h;
        return fail(ALE_LB_EDEVICE, "set-up: %s", hipGetErrorString(e));
    }
    st = upload_clock(h);
    if (st) {
        delete h;
        return st;
    }
    if ((h->flags & ALE_LB_F_PIPELINE) && ncases >= 2) {
        // the case boundary nearest half the node slots
        int best = 1;
        for (int c = 1; c < ncases; ++c)
            if (std::abs(2 * node_off[c] - N) < std::abs(2 * node_off[best] - N)) best = c;
        h->split_case = best;
        h->split_node = node_off[best];
        if (hipStreamCreate(&h->st2) != hipSuccess || hipEventCreateWithFlags(&h->ev_a, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&h->ev_b, hipEventDisableTiming) != hipSuccess) {
            delete h;
            return fail(ALE_LB_EDEVICE, "could not create the second stream of a split batch");
        }
    }
    h->step = 0;
    h->cur = 0;
    *out = h;
    return ALE_LB_OK;
}

}  // namespace

// Checkpoint blob: a header, the per-case times, then the populations and
// macros exactly as stored (node slots in internal order, the storage
// precision; a tile state with its X folded in, as a family switch does).
struct StateBlob {
    char magic[8];       // "ALELBST1"
    int32_t prec;        // bytes per stored value
    int32_t ncases;
    int64_t slots;       // node slots
    int64_t step;
    uint64_t layout;     // hash of the slot -> caller node map
    int64_t bytes;       // of the whole blob
};

namespace {
uint64_t layout_hash(const ale_lb *h)
{
    uint64_t x = 1469598103934665603ull;  // FNV-1a over the slot map
    for (int v : h->perm) {
        x ^= uint64_t(uint32_t(v));
        x *= 1099511628211ull;
    }
    return x;
}

int64_t blob_bytes(const ale_lb *h)
{
    const int64_t rb = h->fp32 ? 4 : 8;
    return int64_t(sizeof(StateBlob)) + 8 * int64_t(h->ncases) + rb * (NPOP + 4) * int64_t(h->N);
}

template <typename R>
int save_blob(ale_lb *h, DevState<R> &s, char *dst)
{
    const size_t np = sizeof(R) * NPOP * size_t(h->N), nm = sizeof(R) * 4 * size_t(h->N);
    if (!tiled(h->sch)) {
        HIP_OK(hipMemcpyAsync(dst, s.pop[h->cur], np, hipMemcpyDeviceToHost, h->st));
    } else {
        // f* = f' + dt A_ia X_a in scratch copies, leaving the handle's state as it is
        R *pop = nullptr, *X = nullptr;
        HIP_OK(h->dmalloc(reinterpret_cast<void **>(&pop), np));
        hipError_t e = h->dmalloc(reinterpret_cast<void **>(&X), sizeof(R) * 2 * size_t(h->N));
        if (e == hipSuccess) e = hipMemcpyAsync(pop, s.pop[h->cur], np, hipMemcpyDeviceToDevice, h->st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(X, s.Xs[h->cur], sizeof(R) * 2 * size_t(h->N), hipMemcpyDeviceToDevice, h->st);
        if (e == hipSuccess) e = launch_fold_x<R>(h->dm, pop, X, h->d_cs, h->st);
        if (e == hipSuccess) e = hipMemcpyAsync(dst, pop, np, hipMemcpyDeviceToHost, h->st);
        if (e == hipSuccess) e = hipStreamSynchronize(h->st);
        h->dmfree(pop);
        h->dmfree(X);
        HIP_OK(e);
    }
    HIP_OK(hipMemcpyAsync(dst + np, s.mac[h->cur], nm, hipMemcpyDeviceToHost, h->st));
    HIP_OK(hipStreamSynchronize(h->st));
    return ALE_LB_OK;
}

template <typename R>
int load_blob(ale_lb *h, DevState<R> &s, const char *src)
{
    const size_t np = sizeof(R) * NPOP * size_t(h->N), nm = sizeof(R) * 4 * size_t(h->N);
    HIP_OK(hipMemcpyAsync(s.pop[h->cur], src, np, hipMemcpyHostToDevice, h->st));
    HIP_OK(hipMemcpyAsync(s.mac[h->cur], src + np, nm, hipMemcpyHostToDevice, h->st));
    HIP_OK(hipStreamSynchronize(h->st));
    return ALE_LB_OK;
}
}  // namespace

// ---- scratch of ale_lb_forces_noalloc ----
// The per-workgroup partial force sums of ale_lb_forces_noalloc live in this
// static array, not in the handle: FORCE_SCRATCH_BLOCKS workgroups of wall
// edges x 6 doubles (192 KiB), one copy per GPU, held until the process ends.
// In host code its name stands for no device address: kernels and copies take
// the address hipGetSymbolAddress gives on each device, looked up once per
// device with that device current.
constexpr int FORCE_SCRATCH_BLOCKS = 4096;
static __device__ __align__(256) double scratch[6 * FORCE_SCRATCH_BLOCKS];

namespace {
constexpr int SCRATCH_DEVICES = 64;
std::mutex g_scratch_mutex;
double *g_scratch[SCRATCH_DEVICES] = {};

// the device address of `scratch` on device dev, which must be current
int scratch_on(int dev, double **out)
{
    if (dev < 0 || dev >= SCRATCH_DEVICES) return fail(ALE_LB_EUNSUPPORTED, "device %d: no scratch slot", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mutex);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(ALE_LB_EDEVICE, "scratch address on device %d: %s", dev, hipGetErrorString(e));
        g_scratch[dev] = static_cast<double *>(p);
    }
    *out = g_scratch[dev];
    return ALE_LB_OK;
}
}  // namespace

extern "C" {

const char *ale_lb_last_error(void) { return g_err.c_str(); }

int ale_lb_create(const ale_lb_mesh_t *mesh, const ale_lb_lattice_t *lattice, const ale_lb_params_t *params,
                  ale_lb_t **out)
{
    return create_impl(mesh, lattice, params, 1, out);
}

int ale_lb_create_batch(const ale_lb_mesh_t *meshes, const ale_lb_params_t *params, int32_t n_cases,
                        const ale_lb_lattice_t *lattice, ale_lb_t **out)
{
    return create_impl(meshes, lattice, params, n_cases, out);
}

void ale_lb_destroy(ale_lb_t *h)
{
    if (h) {
        (void)hipStreamSynchronize(h->st);
        delete h;
    }
}

int ale_lb_step(ale_lb_t *h, int32_t n)
{
    if (!h || n < 0) return fail(ALE_LB_EINVAL, "bad handle or step count");
    if (n == 0) return ALE_LB_OK;
    return h->fp32 ? do_steps(h, h->sf, n, nullptr, nullptr) : do_steps(h, h->sd, n, nullptr, nullptr);
}

int ale_lb_time_kernels(ale_lb_t *h, int32_t n, double *ms, int32_t nk)
{
    if (!h || n <= 0 || !ms || nk < NKERNELS + 1) return fail(ALE_LB_EINVAL, "bad arguments");
    hipEvent_t ev[NKERNELS + 1] = {};
    double acc[NKERNELS + 1] = {};
    int st = ALE_LB_OK;
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            e = nullptr;
            st = fail(ALE_LB_EDEVICE, "could not create the timing events");
            break;
        }
    if (!st) st = h->fp32 ? do_steps(h, h->sf, n, ev, acc) : do_steps(h, h->sd, n, ev, acc);
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    if (st) return st;
    for (int k = 0; k <= NKERNELS; ++k) ms[k] = acc[k] / n;
    return st;
}

int ale_lb_init_fields(ale_lb_t *h, const double *rho, const double *ux, const double *uy, const double *T)
{
    if (!h || !rho || !ux || !uy || !T) return fail(ALE_LB_EINVAL, "null argument");
    const size_t N = h->N;
    std::vector<double> tmp(4 * N, 0.0);
    const double *src[4] = {rho, ux, uy, T};
    for (int c = 0; c < 4; ++c)
        for (size_t k = 0; k < N; ++k) tmp[c * N + k] = h->perm[k] >= 0 ? src[c][h->perm[k]] : 1.0;
    double *d = nullptr;
    HIP_OK(h->dmalloc(reinterpret_cast<void **>(&d), sizeof(double) * 4 * N));
    hipError_t e = hipMemcpyAsync(d, tmp.data(), sizeof(double) * 4 * N, hipMemcpyHostToDevice, h->st);
    if (e == hipSuccess)
        e = h->fp32 ? launch_init<float>(h->dm, h->sf, h->d_cs, d, d + N, d + 2 * N, d + 3 * N, h->cur, h->st)
                    : launch_init<double>(h->dm, h->sd, h->d_cs, d, d + N, d + 2 * N, d + 3 * N, h->cur, h->st);
    if (e == hipSuccess) e = clear_x(h);
    if (e == hipSuccess) e = hipStreamSynchronize(h->st);
    h->dmfree(d);
    HIP_OK(e);
    for (int c = 0; c < h->ncases; ++c) h->t[c] = h->prm[c].t0;
    h->step = 0;
    return upload_clock(h);
}

int ale_lb_get_state(ale_lb_t *h, double *pops, double *macros, double *t, int64_t *step)
{
    if (!h) return fail(ALE_LB_EINVAL, "null handle");
    int st = ALE_LB_OK;
    const bool tile = tiled(h->sch);
    if (pops)
        st = h->fp32 ? fetch_nodes<float>(h, h->sf.pop[h->cur], NPOP, pops, true, tile ? h->sf.Xs[h->cur] : nullptr)
                     : fetch_nodes<double>(h, h->sd.pop[h->cur], NPOP, pops, true, tile ? h->sd.Xs[h->cur] : nullptr);
    if (!st && macros) st = h->fp32 ? fetch_nodes<float>(h, h->sf.mac[h->cur], 4, macros)
                                    : fetch_nodes<double>(h, h->sd.mac[h->cur], 4, macros);
    if (t) *t = h->t[0];
    if (step) *step = h->step;
    return st;
}

int ale_lb_set_state(ale_lb_t *h, const double *pops, const double *macros, double t, int64_t step)
{
    if (!h || !pops || !macros) return fail(ALE_LB_EINVAL, "null argument");
    int st = h->fp32 ? put_nodes<float>(h, pops, NPOP, h->sf.pop[h->cur], true)
                     : put_nodes<double>(h, pops, NPOP, h->sd.pop[h->cur], true);
    if (!st) st = h->fp32 ? put_nodes<float>(h, macros, 4, h->sf.mac[h->cur]) : put_nodes<double>(h, macros, 4, h->sd.mac[h->cur]);
    if (st) return st;
    HIP_OK(clear_x(h));
    for (int c = 0; c < h->ncases; ++c) h->t[c] = t;
    h->step = step;
    return upload_clock(h);
}

int64_t ale_lb_state_bytes(ale_lb_t *h)
{
    if (!h) return int64_t(fail(ALE_LB_EINVAL, "null handle"));
    return blob_bytes(h);
}

int ale_lb_save_state(ale_lb_t *h, void *buf, int64_t bytes)
{
    if (!h || !buf) return fail(ALE_LB_EINVAL, "null argument");
    const int64_t need = blob_bytes(h);
    if (bytes < need) return fail(ALE_LB_EINVAL, "save_state: the blob needs %lld bytes, got %lld", (long long)need,
                                  (long long)bytes);
    char *out = static_cast<char *>(buf);
    StateBlob hd;
    std::memset(&hd, 0, sizeof hd);
    std::memcpy(hd.magic, "ALELBST1", 8);
    hd.prec = h->fp32 ? 4 : 8;
    hd.ncases = h->ncases;
    hd.slots = int64_t(h->N);
    hd.step = h->step;
    hd.layout = layout_hash(h);
    hd.bytes = need;
    std::memcpy(out, &hd, sizeof hd);
    std::memcpy(out + sizeof hd, h->t.data(), 8 * size_t(h->ncases));
    char *arr = out + sizeof hd + 8 * size_t(h->ncases);
    return h->fp32 ? save_blob<float>(h, h->sf, arr) : save_blob<double>(h, h->sd, arr);
}

int ale_lb_load_state(ale_lb_t *h, const void *buf, int64_t bytes)
{
    if (!h || !buf) return fail(ALE_LB_EINVAL, "null argument");
    StateBlob hd;
    if (bytes < int64_t(sizeof hd)) return fail(ALE_LB_EINVAL, "load_state: %lld bytes is no state blob", (long long)bytes);
    std::memcpy(&hd, buf, sizeof hd);
    if (std::memcmp(hd.magic, "ALELBST1", 8) != 0) return fail(ALE_LB_EINVAL, "load_state: not a state blob");
    if (hd.prec != (h->fp32 ? 4 : 8) || hd.ncases != h->ncases || hd.slots != int64_t(h->N) ||
        hd.layout != layout_hash(h) || hd.bytes != blob_bytes(h) || bytes < hd.bytes)
        return fail(ALE_LB_EINVAL, "load_state: the blob was saved by a handle of another precision, mesh or batch");
    const char *in = static_cast<const char *>(buf);
    std::vector<double> t(size_t(h->ncases));
    std::memcpy(t.data(), in + sizeof hd, 8 * size_t(h->ncases));
    for (double v : t)
        if (!std::isfinite(v)) return fail(ALE_LB_EINVAL, "load_state: a case time is not finite");
    const char *arr = in + sizeof hd + 8 * size_t(h->ncases);
    int st = h->fp32 ? load_blob<float>(h, h->sf, arr) : load_blob<double>(h, h->sd, arr);
    if (st) return st;
    HIP_OK(clear_x(h));
    h->t = t;
    h->step = hd.step;
    return upload_clock(h);
}

int ale_lb_get_times(ale_lb_t *h, double *t, int32_t n)
{
    if (!h || !t) return fail(ALE_LB_EINVAL, "null argument");
    for (int c = 0; c < n && c < h->ncases; ++c) t[c] = h->t[c];
    return ALE_LB_OK;
}

int ale_lb_set_times(ale_lb_t *h, const double *t, int32_t n)
{
    if (!h || !t) return fail(ALE_LB_EINVAL, "null argument");
    if (n != h->ncases) return fail(ALE_LB_EINVAL, "set_times needs one time per case (%d, got %d)", h->ncases, n);
    for (int c = 0; c < n; ++c)
        if (!std::isfinite(t[c])) return fail(ALE_LB_EINVAL, "time of case %d is not finite", c);
    for (int c = 0; c < n; ++c) h->t[c] = t[c];
    return upload_clock(h);
}

int ale_lb_get_fields(ale_lb_t *h, double *rho, double *ux, double *uy, double *T, int32_t on_device)
{
    if (!h) return fail(ALE_LB_EINVAL, "null handle");
    const size_t N = h->N;
    double *dst[4] = {rho, ux, uy, T};
    if (on_device) {
        double *d = nullptr;
        HIP_OK(h->dmalloc(reinterpret_cast<void **>(&d), sizeof(double) * 4 * N));
        hipError_t e = h->fp32 ? launch_convert<float>(h->sf.mac[h->cur], d, N, 4, h->st)
                               : launch_convert<double>(h->sd.mac[h->cur], d, N, 4, h->st);
        for (int c = 0; c < 4 && e == hipSuccess; ++c)
            if (dst[c]) e = hipMemcpyAsync(dst[c], d + c * N, sizeof(double) * N, hipMemcpyDeviceToDevice, h->st);
        if (e == hipSuccess) e = hipStreamSynchronize(h->st);
        h->dmfree(d);
        HIP_OK(e);
        return ALE_LB_OK;
    }
    const size_t M = h->Ncaller;
    std::vector<double> mac(4 * M);
    int st = ale_lb_get_state(h, nullptr, mac.data(), nullptr, nullptr);
    if (st) return st;
    for (int c = 0; c < 4; ++c)
        if (dst[c]) std::memcpy(dst[c], mac.data() + c * M, sizeof(double) * M);
    return ALE_LB_OK;
}

int ale_lb_get_streamed(ale_lb_t *h, double *pops, int32_t *miss_wall, int32_t *miss_far)
{
    if (!h) return fail(ALE_LB_EINVAL, "null handle");
    if (pops && tiled(h->sch) && !(h->flags & ALE_LB_F_KEEP_MASKS))
        return fail(ALE_LB_EINVAL, "tile schedules record the streamed populations only with ALE_LB_F_KEEP_MASKS");
    int st = ALE_LB_OK;
    if (pops)
        st = h->fp32 ? fetch_nodes<float>(h, h->sf.ft, NPOP, pops, true) : fetch_nodes<double>(h, h->sd.ft, NPOP, pops, true);
    if (st) return st;
    if (miss_wall || miss_far) {
        int *dmask = h->fp32 ? h->sf.mask : h->sd.mask;
        if (!dmask) return fail(ALE_LB_EINVAL, "missing masks need ALE_LB_F_KEEP_MASKS at create");
        std::vector<int> m(h->N);
        HIP_OK(hipMemcpyAsync(m.data(), dmask, sizeof(int) * h->N, hipMemcpyDeviceToHost, h->st));
        HIP_OK(hipStreamSynchronize(h->st));
        for (int k = 0; k < h->N; ++k) {
            if (h->perm[k] < 0) continue;
            if (miss_wall) miss_wall[h->perm[k]] = m[k] & 0xffff;
            if (miss_far) miss_far[h->perm[k]] = (m[k] >> 16) & 0xffff;
        }
    }
    return ALE_LB_OK;
}

int ale_lb_get_correction(ale_lb_t *h, double *W, double *Xa)
{
    if (!h) return fail(ALE_LB_EINVAL, "null handle");
    int st = ALE_LB_OK;
    if (W) st = h->fp32 ? fetch_nodes<float>(h, h->sf.W, 2, W) : fetch_nodes<double>(h, h->sd.W, 2, W);
    const bool tile = tiled(h->sch);
    if (Xa && !tile && !(h->flags & ALE_LB_F_KEEP_MASKS))
        return fail(ALE_LB_EINVAL, "one-wave schedules record X only with ALE_LB_F_KEEP_MASKS");
    if (!st && Xa)
        st = h->fp32 ? fetch_nodes<float>(h, tile ? h->sf.Xs[h->cur] : h->sf.Xc, 2, Xa)
                     : fetch_nodes<double>(h, tile ? h->sd.Xs[h->cur] : h->sd.Xc, 2, Xa);
    return st;
}

int ale_lb_move_mesh(ale_lb_t *h, double t, double *x, double *Jinv, double *detJ, double *vg, int32_t on_device)
{
    if (!h) return fail(ALE_LB_EINVAL, "null handle");
    const size_t N = h->N;
    std::vector<double> tc(h->ncases, t);
    int err = 0;
    HIP_OK(hipMemcpyAsync(h->d_tcase, tc.data(), sizeof(double) * h->ncases, hipMemcpyHostToDevice, h->st));
    HIP_OK(hipMemcpyAsync(h->d_err, &err, sizeof(int), hipMemcpyHostToDevice, h->st));
    if (on_device) {
        HIP_OK(launch_move_mesh(h->dm, h->d_cs, h->d_tcase, x, Jinv, detJ, vg, h->d_err, h->st));
    } else {
        double *d = nullptr;
        HIP_OK(h->dmalloc(reinterpret_cast<void **>(&d), sizeof(double) * 9 * N));
        std::vector<double> tmp(9 * N);
        hipError_t e = launch_move_mesh(h->dm, h->d_cs, h->d_tcase, d, d + 2 * N, d + 6 * N, d + 7 * N, h->d_err, h->st);
        if (e == hipSuccess) e = hipMemcpyAsync(tmp.data(), d, sizeof(double) * 9 * N, hipMemcpyDeviceToHost, h->st);
        if (e == hipSuccess) e = hipStreamSynchronize(h->st);
        h->dmfree(d);
        HIP_OK(e);
        for (size_t k = 0; k < N; ++k) {
            if (h->perm[k] < 0) continue;
            const size_t a = h->perm[k];
            if (x) { x[2 * a] = tmp[2 * k]; x[2 * a + 1] = tmp[2 * k + 1]; }
            if (Jinv) for (int q = 0; q < 4; ++q) Jinv[4 * a + q] = tmp[2 * N + 4 * k + q];
            if (detJ) detJ[a] = tmp[6 * N + k];
            if (vg) { vg[2 * a] = tmp[7 * N + 2 * k]; vg[2 * a + 1] = tmp[7 * N + 2 * k + 1]; }
        }
    }
    HIP_OK(hipMemcpyAsync(&err, h->d_err, sizeof(int), hipMemcpyDeviceToHost, h->st));
    HIP_OK(hipStreamSynchronize(h->st));
    const int zero = 0;
    HIP_OK(hipMemcpyAsync(h->d_err, &zero, sizeof(int), hipMemcpyHostToDevice, h->st));
    HIP_OK(hipStreamSynchronize(h->st));
    if (err & ERR_JAC) return fail(ALE_LB_EJAC, "mapping Jacobian det <= 0 at t = %g", t);
    return ALE_LB_OK;
}

int ale_lb_forces_batch(ale_lb_t *h, ale_lb_forces_t *out, int32_t n)
{
    if (!h || !out || n < 1) return fail(ALE_LB_EINVAL, "bad arguments");
    std::vector<double> F(6 * size_t(h->ncases), 0.0);
    if (h->force_blocks > 0) {
        hipError_t e = h->fp32 ? launch_forces<float>(h->dm, h->sf.mac[h->cur], h->d_cs, clock_of(h, h->cur ^ 1), h->d_part,
                                                      h->force_blocks, h->d_case_blocks, h->d_fout, h->st)
                               : launch_forces<double>(h->dm, h->sd.mac[h->cur], h->d_cs, clock_of(h, h->cur ^ 1), h->d_part,
                                                       h->force_blocks, h->d_case_blocks, h->d_fout, h->st);
        HIP_OK(e);
        HIP_OK(hipMemcpyAsync(F.data(), h->d_fout, sizeof(double) * 6 * h->ncases, hipMemcpyDeviceToHost, h->st));
        HIP_OK(hipStreamSynchronize(h->st));
    }
    for (int c = 0; c < n && c < h->ncases; ++c) {
        const double *f = &F[6 * c];
        const ale_lb_params_t &p = h->prm[c];
        ale_lb_forces_t &o = out[c];
        o.F_p[0] = f[0];
        o.F_p[1] = f[1];
        o.F_v[0] = f[2];
        o.F_v[1] = f[3];
        o.M_p = f[4];
        o.M_v = f[5];
        const double U2 = p.u_inf[0] * p.u_inf[0] + p.u_inf[1] * p.u_inf[1];
        const double qc = 0.5 * p.rho_inf * U2 * p.chord;
        o.cl = qc > 0 ? (f[1] + f[3]) / qc : 0.0;
        o.cd = qc > 0 ? (f[0] + f[2]) / qc : 0.0;
        o.cm = qc > 0 ? (f[4] + f[5]) / (qc * p.chord) : 0.0;
        o.t = h->t[c];
    }
    return ALE_LB_OK;
}

int ale_lb_forces(ale_lb_t *h, ale_lb_forces_t *out) { return ale_lb_forces_batch(h, out, 1); }

int ale_lb_forces_noalloc(ale_lb_t *h, double *out_dev, int32_t n)
{
    if (!h || !out_dev) return fail(ALE_LB_EINVAL, "forces_noalloc: null argument");
    if (n < h->ncases) return fail(ALE_LB_EINVAL, "forces_noalloc: room for %d cases, the batch has %d", n, h->ncases);
    if (h->force_blocks > FORCE_SCRATCH_BLOCKS)
        return fail(ALE_LB_EINVAL, "forces_noalloc: the wall edges take %d workgroups, the scratch holds %d",
                    h->force_blocks, FORCE_SCRATCH_BLOCKS);
    int dev = -1;
    HIP_OK(hipGetDevice(&dev));
    if (dev != h->device)
        return fail(ALE_LB_EINVAL, "forces_noalloc: device %d is current, the handle's is %d", dev, h->device);
    double *part = nullptr;
    const int st = scratch_on(dev, &part);
    if (st) return st;
    HIP_OK(h->fp32 ? launch_forces<float>(h->dm, h->sf.mac[h->cur], h->d_cs, clock_of(h, h->cur ^ 1), part,
                                          h->force_blocks, h->d_case_blocks, out_dev, h->st)
                   : launch_forces<double>(h->dm, h->sd.mac[h->cur], h->d_cs, clock_of(h, h->cur ^ 1), part,
                                           h->force_blocks, h->d_case_blocks, out_dev, h->st));
    return ALE_LB_OK;
}

int ale_lb_set_schedule(ale_lb_t *h, int32_t waves, int32_t rings, int32_t node_block, int32_t lds_limit,
                        int32_t groups)
{
    if (!h || lds_limit < 0) return fail(ALE_LB_EINVAL, "bad arguments");
    h->lds_limit = lds_limit;
    return set_schedule(h, Schedule{waves, rings, node_block, groups == 0 ? 1 : groups});
}

int ale_lb_autotune(ale_lb_t *h, int32_t reps, int32_t *choice, double *ms)
{
    if (!h || reps < 0) return fail(ALE_LB_EINVAL, "bad arguments");
    const TuneKey key = tune_key(h);
    int st = ALE_LB_OK;
    int cached = 0;
    Schedule found{};
    {
        std::lock_guard<std::mutex> lk(g_tune_mutex);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            found = it->second;
            cached = 1;
        }
    }
    if (ms) *ms = 0.0;
    if (cached && reps > 0) {
        h->lds_limit = 0;
        st = set_schedule(h, found);
    } else if (reps > 0) {
        h->lds_limit = 0;
        st = h->fp32 ? autotune(h, h->sf, reps, ms) : autotune(h, h->sd, reps, ms);
        if (!st) {
            std::lock_guard<std::mutex> lk(g_tune_mutex);
            g_tune_cache[key] = h->sch;
        }
    } else {
        // reps == 0: forget the cached choice of this mesh-size bucket
        std::lock_guard<std::mutex> lk(g_tune_mutex);
        g_tune_cache.erase(key);
    }
    if (choice) {
        choice[0] = h->sch.waves;
        choice[1] = h->sch.rings;
        choice[2] = h->sch.node_block;
        choice[3] = cached;
        choice[4] = tiled(h->sch) ? h->tile_overflow : 0;
        choice[5] = h->sch.groups;
    }
    return st;
}

int ale_lb_info(ale_lb_t *h, int64_t *out, int32_t n)
{
    if (!h || !out) return fail(ALE_LB_EINVAL, "null argument");
    const bool tl = tiled(h->sch);
    const int64_t v[12] = {h->Ncaller, h->E, h->NWE, h->NW, int64_t(h->dev_bytes), h->fp32 ? 4 : 8, h->ncases, h->N,
                           tl ? h->tile_overflow : 0, tl ? h->ta.pn_max : 0, tl ? h->ta.pe_max : 0,
                           tl ? int64_t(tile_lds_bytes(h->ta.pe_max, h->ta.pn_max, h->fp32 ? 4 : 8, h->ta.tile)) : 0};
    for (int k = 0; k < n && k < 12; ++k) out[k] = v[k];
    return ALE_LB_OK;
}

int ale_lb_node_order(ale_lb_t *h, int32_t *perm)
{
    if (!h || !perm) return fail(ALE_LB_EINVAL, "null argument");
    int k = 0;
    for (int s = 0; s < h->N; ++s)
        if (h->perm[s] >= 0) perm[k++] = h->perm[s];
    return ALE_LB_OK;
}

}  // extern "C"
