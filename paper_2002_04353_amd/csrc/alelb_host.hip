// Host runtime of the ALE lattice-Boltzmann library: the C-ABI declared in
// include/alelb.h.  Builds the static mesh data (element frames and affine
// inverses, owner map, wall normals and points B), reorders nodes and
// elements along a Morton curve, owns the device buffers and enqueues the
// gfx950 kernels of alelb_kernels.hip on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
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

uint64_t spread21(uint64_t v)
{
    v &= 0x1fffff;
    v = (v | (v << 32)) & 0x1f00000000ffffULL;
    v = (v | (v << 16)) & 0x1f0000ff0000ffULL;
    v = (v | (v << 8)) & 0x100f00f00f00f00fULL;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ULL;
    v = (v | (v << 2)) & 0x1249249249249249ULL;
    return v;
}

// Morton order of a point set over its bounding box (ties by index)
std::vector<int> morton_order(const std::vector<double> &xy)
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
        key[i] = spread21(qx) | (spread21(qy) << 1);
    }
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return key[a] < key[b]; });
    return ord;
}

struct HostMesh {
    int N = 0, E = 0;
    std::vector<double> X;       // [2N]
    std::vector<int> elem, nbr;  // [6E], [3E]
    std::vector<int8_t> psh;     // [3E]
    double L[2] = {0, 0};
    std::vector<int> wedge;      // [2 NWE]
    // derived, input order
    std::vector<double> ev;      // [6E] vertex coordinates in each element frame
    std::vector<double> A;       // [4E]
    std::vector<double> area;
    std::vector<int> owner, oslot;
    std::vector<double> opos;    // [2N]
};

// walk on the host (used once per wall node to locate its point B)
int host_walk(const HostMesh &h, int e, double P[2], double l[3])
{
    for (int it = 0; it < WALK_CAP; ++it) {
        const double *v = &h.ev[6 * e];
        const double *A = &h.A[4 * e];
        const double dx = P[0] - v[0], dy = P[1] - v[1];
        l[1] = A[0] * dx + A[1] * dy;
        l[2] = A[2] * dx + A[3] * dy;
        l[0] = 1.0 - l[1] - l[2];
        int k = 0;
        double mn = l[0];
        if (l[1] < mn) { k = 1; mn = l[1]; }
        if (l[2] < mn) { k = 2; mn = l[2]; }
        if (mn >= -TAU_LOC) return e;
        const int n = h.nbr[3 * e + k];
        if (n < 0) return n;
        const int code = h.psh[3 * e + k];
        if (code != 0) {
            P[0] += double((code + 4) % 3 - 1) * h.L[0];
            P[1] += double((code + 4) / 3 - 1) * h.L[1];
        }
        e = n;
    }
    return -4;
}

struct DeviceBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct ale_lb {
    ale_lb_params_t prm{};
    ale_lb_lattice_t lat{};
    HostMesh hm;
    int N = 0, E = 0, NW = 0, NWE = 0;
    std::vector<int> perm;   // internal -> caller node
    std::vector<int> iperm;  // caller -> internal node
    hipStream_t st = nullptr;
    bool fp32 = false;
    std::vector<DeviceBuf> bufs;
    size_t dev_bytes = 0;
    DevMesh dm{};
    DevState<float> sf{};
    DevState<double> sd{};
    Phys ph{};
    Motion mo{};
    int cur = 0;
    double t = 0.0;
    int64_t step = 0;
    int *d_err = nullptr;
    double *d_part = nullptr;
    double *d_fout = nullptr;
    int force_blocks = 1;

    void *alloc(size_t bytes, int *status)
    {
        void *p = nullptr;
        if (bytes == 0) bytes = 8;
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            *status = fail(e == hipErrorOutOfMemory ? ALE_LB_ENOMEM : ALE_LB_EDEVICE, "hipMalloc(%zu): %s", bytes,
                           hipGetErrorString(e));
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
    ~ale_lb()
    {
        for (auto &b : bufs) (void)hipFree(b.p);
    }
};

namespace {

int validate_and_derive(HostMesh &h, std::string &why)
{
    const int N = h.N, E = h.E;
    char buf[256];
    for (int e = 0; e < E; ++e)
        for (int k = 0; k < 6; ++k)
            if (h.elem[6 * e + k] < 0 || h.elem[6 * e + k] >= N) {
                snprintf(buf, sizeof buf, "element %d references node %d out of range", e, h.elem[6 * e + k]);
                why = buf;
                return ALE_LB_EMESH;
            }
    h.ev.resize(6 * size_t(E));
    h.A.resize(4 * size_t(E));
    h.area.resize(E);
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
    for (int e = 0; e < E; ++e)
        for (int k = 0; k < 3; ++k) {
            const int n = h.nbr[3 * e + k];
            if (n >= E || n < -2) {
                snprintf(buf, sizeof buf, "neighbour of element %d out of range", e);
                why = buf;
                return ALE_LB_EMESH;
            }
            if (n >= 0 && h.nbr[3 * n] != e && h.nbr[3 * n + 1] != e && h.nbr[3 * n + 2] != e) {
                snprintf(buf, sizeof buf, "neighbours of elements %d and %d are not symmetric", e, n);
                why = buf;
                return ALE_LB_EMESH;
            }
            const int c = h.psh[3 * e + k];
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
        for (int k = 0; k < 6; ++k) {
            const int a = h.elem[6 * e + k];
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
        const int e = h.owner[a], k = h.oslot[a];
        const double *v = &h.ev[6 * e];
        if (k < 3) {
            h.opos[2 * a] = v[2 * k];
            h.opos[2 * a + 1] = v[2 * k + 1];
        } else {
            const int k1 = (k - 3 + 1) % 3, k2 = (k - 3 + 2) % 3;
            h.opos[2 * a] = 0.5 * (v[2 * k1] + v[2 * k2]);
            h.opos[2 * a + 1] = 0.5 * (v[2 * k1 + 1] + v[2 * k2 + 1]);
        }
    }
    return ALE_LB_OK;
}

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
    if (st) return st;
    HIP_OK(hipMemset(s.ft, 0, sizeof(R) * NPOP * N));
    HIP_OK(hipMemset(s.W, 0, sizeof(R) * 2 * N));
    HIP_OK(hipMemset(s.Xc, 0, sizeof(R) * 2 * N));
    s.mask = nullptr;
    if (h->prm.flags & ALE_LB_F_KEEP_MASKS) {
        s.mask = static_cast<int *>(h->alloc(sizeof(int) * N, &st));
        if (st) return st;
        HIP_OK(hipMemset(s.mask, 0, sizeof(int) * N));
    }
    s.err = h->d_err;
    s.finf = static_cast<R *>(h->alloc(sizeof(R) * NPOP, &st));
    s.wl_count = static_cast<int *>(h->alloc(sizeof(int), &st));
    s.wl_node = static_cast<int *>(h->alloc(sizeof(int) * N, &st));
    s.wl_mask = static_cast<int *>(h->alloc(sizeof(int) * N, &st));
    if (st) return st;
    HIP_OK(hipMemset(s.wl_count, 0, sizeof(int)));
    return ALE_LB_OK;
}

int check_err(ale_lb *h)
{
    int err = 0;
    HIP_OK(hipMemcpyAsync(&err, h->d_err, sizeof(int), hipMemcpyDeviceToHost, h->st));
    HIP_OK(hipStreamSynchronize(h->st));
    if (err) {
        HIP_OK(hipMemsetAsync(h->d_err, 0, sizeof(int), h->st));
        HIP_OK(hipStreamSynchronize(h->st));
        if (err & ERR_JAC) return fail(ALE_LB_EJAC, "mapping Jacobian det <= 0 (step %lld)", (long long)h->step);
        if (err & ERR_LOCATE) return fail(ALE_LB_ELOCATE, "element walk exceeded %d steps (step %lld)", WALK_CAP, (long long)h->step);
        if (err & ERR_NONFINITE) return fail(ALE_LB_ENONFINITE, "non-finite populations (step %lld)", (long long)h->step);
    }
    return ALE_LB_OK;
}

template <typename R>
int do_steps(ale_lb *h, DevState<R> &s, int n, hipEvent_t *ev, double *ms)
{
    for (int k = 0; k < n; ++k) {
        StepArgs<R> a;
        a.m = h->dm;
        a.s = s;
        a.ph = h->ph;
        a.mo = h->mo;
        a.th = motion_time(h->mo, h->t + 0.5 * h->prm.dt);
        a.t1 = motion_time(h->mo, h->t + h->prm.dt);
        a.cur = h->cur;
        HIP_OK(launch_step<R>(a, h->st, ev));
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
        h->cur ^= 1;
        h->t = h->t + h->prm.dt;
        h->step += 1;
        if (h->prm.check_every > 0 && (k + 1) % h->prm.check_every == 0) {
            const int st = check_err(h);
            if (st) return st;
        }
    }
    return check_err(h);
}

template <typename R>
int get_state_t(ale_lb *h, DevState<R> &s, const R *src_pop, const R *src_mac, double *pops, double *macros)
{
    const size_t N = h->N;
    std::vector<double> tmp;
    double *d = nullptr;
    HIP_OK(hipMalloc(&d, sizeof(double) * NPOP * N));
    auto fetch = [&](const R *src, size_t cnt, double *out) -> int {
        HIP_OK(launch_convert<R>(src, d, N, int(cnt), h->st));
        tmp.resize(cnt * N);
        HIP_OK(hipMemcpyAsync(tmp.data(), d, sizeof(double) * cnt * N, hipMemcpyDeviceToHost, h->st));
        HIP_OK(hipStreamSynchronize(h->st));
        for (size_t c = 0; c < cnt; ++c)
            for (size_t k = 0; k < N; ++k) out[c * N + h->perm[k]] = tmp[c * N + k];
        return ALE_LB_OK;
    };
    int st = ALE_LB_OK;
    if (pops && src_pop) st = fetch(src_pop, NPOP, pops);
    if (!st && macros && src_mac) st = fetch(src_mac, 4, macros);
    (void)hipFree(d);
    (void)s;
    return st;
}

template <typename R>
int set_state_t(ale_lb *h, DevState<R> &s, const double *pops, const double *macros)
{
    const size_t N = h->N;
    std::vector<double> tmp(NPOP * N);
    double *d = nullptr;
    HIP_OK(hipMalloc(&d, sizeof(double) * NPOP * N));
    auto put = [&](const double *in, size_t cnt, R *dst) -> int {
        for (size_t c = 0; c < cnt; ++c)
            for (size_t k = 0; k < N; ++k) tmp[c * N + k] = in[c * N + h->perm[k]];
        HIP_OK(hipMemcpyAsync(d, tmp.data(), sizeof(double) * cnt * N, hipMemcpyHostToDevice, h->st));
        HIP_OK(launch_convert_back<R>(d, dst, N, int(cnt), h->st));
        HIP_OK(hipStreamSynchronize(h->st));
        return ALE_LB_OK;
    };
    int st = put(pops, NPOP, s.pop[h->cur]);
    if (!st) st = put(macros, 4, s.mac[h->cur]);
    (void)hipFree(d);
    return st;
}

}  // namespace

extern "C" {

const char *ale_lb_last_error(void) { return g_err.c_str(); }

int ale_lb_create(const ale_lb_mesh_t *mesh, const ale_lb_lattice_t *lattice, const ale_lb_params_t *params,
                  ale_lb_t **out)
{
    if (!mesh || !lattice || !params || !out) return fail(ALE_LB_EINVAL, "null argument");
    *out = nullptr;
    if (lattice->Q != 9) return fail(ALE_LB_EUNSUPPORTED, "only the D2Q9 lattice is supported (Q = %d)", lattice->Q);
    if (lattice->shift[0] != 0.0 || lattice->shift[1] != 0.0)
        return fail(ALE_LB_EUNSUPPORTED, "shifted lattices are not supported");
    if (!(lattice->gamma > 1.0) || !(lattice->Pr > 0.0)) return fail(ALE_LB_EINVAL, "gamma must exceed 1 and Pr be positive");
    if (mesh->n_nodes <= 0 || mesh->n_elems <= 0 || !mesh->X || !mesh->elem || !mesh->nbr)
        return fail(ALE_LB_EINVAL, "empty mesh");
    if (!(params->dt > 0.0) || !(params->mu >= 0.0)) return fail(ALE_LB_EINVAL, "dt must be positive, mu non-negative");
    if (params->precision != ALE_LB_FP64 && params->precision != ALE_LB_FP32)
        return fail(ALE_LB_EINVAL, "unknown precision %d", params->precision);
    if (params->motion < 0 || params->motion > 3) return fail(ALE_LB_EINVAL, "unknown motion law %d", params->motion);
    if (mesh->n_wall_edges < 0 || (mesh->n_wall_edges > 0 && !mesh->wall_edges))
        return fail(ALE_LB_EINVAL, "bad wall-edge list");

    ale_lb *h = new ale_lb();
    h->prm = *params;
    h->lat = *lattice;
    h->st = static_cast<hipStream_t>(params->stream);
    h->fp32 = params->precision == ALE_LB_FP32;
    HostMesh &hm = h->hm;
    hm.N = h->N = mesh->n_nodes;
    hm.E = h->E = mesh->n_elems;
    hm.X.assign(mesh->X, mesh->X + 2 * size_t(hm.N));
    hm.elem.assign(mesh->elem, mesh->elem + 6 * size_t(hm.E));
    hm.nbr.assign(mesh->nbr, mesh->nbr + 3 * size_t(hm.E));
    hm.psh.assign(3 * size_t(hm.E), 0);
    if (mesh->pshift) hm.psh.assign(mesh->pshift, mesh->pshift + 3 * size_t(hm.E));
    hm.L[0] = mesh->period[0];
    hm.L[1] = mesh->period[1];
    h->NWE = mesh->n_wall_edges;
    if (h->NWE > 0) hm.wedge.assign(mesh->wall_edges, mesh->wall_edges + 2 * size_t(h->NWE));
    std::string why;
    int st = validate_and_derive(hm, why);
    if (st) {
        delete h;
        return fail(st, "%s", why.c_str());
    }
    const int N = h->N, E = h->E;
    // wall nodes, computational into-fluid normals, points B (Sec. IV.A)
    std::vector<int> wid(N, -1);
    std::vector<double> nacc(2 * size_t(N), 0.0);
    int nw = 0;
    for (int w = 0; w < h->NWE; ++w) {
        const int e = hm.wedge[2 * w], k = hm.wedge[2 * w + 1];
        if (e < 0 || e >= E || k < 0 || k > 2 || hm.nbr[3 * e + k] != -1) {
            delete h;
            return fail(ALE_LB_EMESH, "wall edge %d is not a wall-tagged element edge", w);
        }
        const double *v = &hm.ev[6 * e];
        const int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
        const double dx = v[2 * k2] - v[2 * k1], dy = v[2 * k2 + 1] - v[2 * k1 + 1];
        const double L = std::sqrt(dx * dx + dy * dy);
        const int nodes[3] = {hm.elem[6 * e + k1], hm.elem[6 * e + k2], hm.elem[6 * e + 3 + k]};
        for (int a : nodes) {
            if (wid[a] < 0) wid[a] = nw++;
            nacc[2 * a] += -dy / L;
            nacc[2 * a + 1] += dx / L;
        }
    }
    h->NW = nw;
    std::vector<int> bel_in(std::max(nw, 1), 0);
    std::vector<double> blam(3 * size_t(std::max(nw, 1)), 0.0);
    for (int a = 0; a < N; ++a) {
        const int w = wid[a];
        if (w < 0) continue;
        const double L = std::sqrt(nacc[2 * a] * nacc[2 * a] + nacc[2 * a + 1] * nacc[2 * a + 1]);
        double B[2] = {hm.opos[2 * a] + params->dt * (nacc[2 * a] / L),
                       hm.opos[2 * a + 1] + params->dt * (nacc[2 * a + 1] / L)};
        double l[3];
        const int eb = host_walk(hm, hm.owner[a], B, l);
        if (eb < 0) {
            delete h;
            return fail(ALE_LB_EMESH, "point B of wall node %d lies outside the mesh", a);
        }
        bel_in[w] = eb;
        blam[3 * w] = l[0];
        blam[3 * w + 1] = l[1];
        blam[3 * w + 2] = l[2];
    }

    // Morton order of nodes (canonical coordinates) and elements (frame centroids)
    h->perm = morton_order(hm.X);
    h->iperm.assign(N, 0);
    for (int k = 0; k < N; ++k) h->iperm[h->perm[k]] = k;
    std::vector<double> cen(2 * size_t(E));
    for (int e = 0; e < E; ++e) {
        const double *v = &hm.ev[6 * e];
        for (int d = 0; d < 2; ++d) {
            double c = (v[d] + v[2 + d] + v[4 + d]) / 3.0;
            if (hm.L[d] > 0.0) c = c - hm.L[d] * std::floor(c / hm.L[d]);
            cen[2 * e + d] = c;
        }
    }
    const std::vector<int> eperm = morton_order(cen);
    std::vector<int> eiperm(E);
    for (int k = 0; k < E; ++k) eiperm[eperm[k]] = k;

    // device mesh arrays in internal order
    std::vector<double2> X(N);
    std::vector<int> own(N), widv(N);
    std::vector<uint8_t> oinfo(N);
    for (int k = 0; k < N; ++k) {
        const int a = h->perm[k];
        X[k] = make_double2(hm.X[2 * a], hm.X[2 * a + 1]);
        own[k] = eiperm[hm.owner[a]];
        int sx = 0, sy = 0;
        if (hm.L[0] > 0.0) sx = int(std::lround((hm.opos[2 * a] - hm.X[2 * a]) / hm.L[0]));
        if (hm.L[1] > 0.0) sy = int(std::lround((hm.opos[2 * a + 1] - hm.X[2 * a + 1]) / hm.L[1]));
        if (sx < -1 || sx > 1 || sy < -1 || sy > 1) {
            delete h;
            return fail(ALE_LB_EMESH, "node %d lies more than one period from its owner element", a);
        }
        oinfo[k] = uint8_t(hm.oslot[a] | (((sx + 1) + 3 * (sy + 1)) << 3));
        widv[k] = wid[a];
    }
    std::vector<ElemRec> el(E);
    for (int k = 0; k < E; ++k) {
        const int e = eperm[k];
        ElemRec &r = el[k];
        r.v0 = make_double2(hm.ev[6 * e], hm.ev[6 * e + 1]);
        r.a01 = make_double2(hm.A[4 * e], hm.A[4 * e + 1]);
        r.a23 = make_double2(hm.A[4 * e + 2], hm.A[4 * e + 3]);
        for (int s = 0; s < 6; ++s) r.n[s] = h->iperm[hm.elem[6 * e + s]];
        r.pad[0] = r.pad[1] = 0;
        int nb[3];
        unsigned codes = 0;
        for (int q = 0; q < 3; ++q) {
            const int n = hm.nbr[3 * e + q];
            nb[q] = n >= 0 ? eiperm[n] : n;
            codes |= unsigned(hm.psh[3 * e + q] + 4) << (4 * q);
        }
        r.nb = make_int4(nb[0], nb[1], nb[2], int(codes));
    }
    std::vector<int> bel(std::max(nw, 1));
    for (int w = 0; w < nw; ++w) bel[w] = eiperm[bel_in[w]];
    std::vector<int2> wedge(std::max(h->NWE, 1));
    std::vector<double4> wxy(std::max(h->NWE, 1));
    for (int w = 0; w < h->NWE; ++w) {
        const int e = hm.wedge[2 * w], k = hm.wedge[2 * w + 1];
        wedge[w] = make_int2(eiperm[e], k);
        const double *v = &hm.ev[6 * e];
        const int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
        wxy[w] = make_double4(v[2 * k1], v[2 * k1 + 1], v[2 * k2], v[2 * k2 + 1]);
    }

    st = ALE_LB_OK;
    DevMesh &dm = h->dm;
    dm.N = N;
    dm.E = E;
    dm.NW = nw;
    dm.NWE = h->NWE;
    dm.wall_sides = int(std::count(hm.nbr.begin(), hm.nbr.end(), -1));
    dm.Lx = hm.L[0];
    dm.Ly = hm.L[1];
    dm.X = h->upload(X, &st);
    dm.own = h->upload(own, &st);
    dm.oinfo = h->upload(oinfo, &st);
    dm.wid = h->upload(widv, &st);
    dm.el = h->upload(el, &st);
    dm.bel = h->upload(bel, &st);
    dm.blam = h->upload(blam, &st);
    dm.wedge = h->upload(wedge, &st);
    dm.wxy = h->upload(wxy, &st);
    h->d_err = static_cast<int *>(h->alloc(sizeof(int), &st));
    h->force_blocks = std::max(1, (h->NWE + BLOCK - 1) / BLOCK);
    h->d_part = static_cast<double *>(h->alloc(sizeof(double) * 6 * h->force_blocks, &st));
    h->d_fout = static_cast<double *>(h->alloc(sizeof(double) * 8, &st));
    if (st) {
        delete h;
        return st;
    }
    if (hipMemset(h->d_err, 0, sizeof(int)) != hipSuccess) {
        delete h;
        return fail(ALE_LB_EDEVICE, "hipMemset failed");
    }
    st = h->fp32 ? alloc_state(h, h->sf) : alloc_state(h, h->sd);
    if (st) {
        delete h;
        return st;
    }
    Phys &ph = h->ph;
    ph.dt = params->dt;
    ph.mu = params->mu;
    ph.gamma = lattice->gamma;
    ph.Pr = lattice->Pr;
    ph.Cv = 1.0 / (lattice->gamma - 1.0);
    ph.Cp = ph.Cv + 1.0;
    ph.rho_inf = params->rho_inf;
    ph.ux_inf = params->u_inf[0];
    ph.uy_inf = params->u_inf[1];
    ph.T_inf = params->T_inf;
    ph.chord = params->chord;
    ph.refx = params->ref_point[0];
    ph.refy = params->ref_point[1];
    ph.flags = params->flags;
    h->mo.kind = params->motion;
    for (int k = 0; k < 12; ++k) h->mo.p[k] = params->motion_p[k];
    h->t = params->t0;
    h->step = 0;
    h->cur = 0;
    {
        hipError_t e = h->fp32 ? launch_freestream<float>(ph, h->sf.finf, h->st)
                               : launch_freestream<double>(ph, h->sd.finf, h->st);
        if (e == hipSuccess) e = hipStreamSynchronize(h->st);
        if (e != hipSuccess) {
            delete h;
            return fail(ALE_LB_EDEVICE, "free-stream equilibrium: %s", hipGetErrorString(e));
        }
    }
    *out = h;
    return ALE_LB_OK;
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
    hipEvent_t ev[NKERNELS + 1];
    for (auto &e : ev) HIP_OK(hipEventCreate(&e));
    double acc[NKERNELS + 1] = {0, 0, 0, 0, 0};
    const int st = h->fp32 ? do_steps(h, h->sf, n, ev, acc) : do_steps(h, h->sd, n, ev, acc);
    for (auto &e : ev) (void)hipEventDestroy(e);
    for (int k = 0; k <= NKERNELS; ++k) ms[k] = acc[k] / n;
    return st;
}

int ale_lb_init_fields(ale_lb_t *h, const double *rho, const double *ux, const double *uy, const double *T)
{
    if (!h || !rho || !ux || !uy || !T) return fail(ALE_LB_EINVAL, "null argument");
    const size_t N = h->N;
    std::vector<double> tmp(4 * N);
    const double *src[4] = {rho, ux, uy, T};
    for (int c = 0; c < 4; ++c)
        for (size_t k = 0; k < N; ++k) tmp[c * N + k] = src[c][h->perm[k]];
    double *d = nullptr;
    HIP_OK(hipMalloc(&d, sizeof(double) * 4 * N));
    HIP_OK(hipMemcpyAsync(d, tmp.data(), sizeof(double) * 4 * N, hipMemcpyHostToDevice, h->st));
    hipError_t e = h->fp32 ? launch_init<float>(h->dm, h->sf, h->ph, d, d + N, d + 2 * N, d + 3 * N, h->cur, h->st)
                           : launch_init<double>(h->dm, h->sd, h->ph, d, d + N, d + 2 * N, d + 3 * N, h->cur, h->st);
    HIP_OK(e);
    HIP_OK(hipStreamSynchronize(h->st));
    (void)hipFree(d);
    h->t = h->prm.t0;
    h->step = 0;
    return ALE_LB_OK;
}

int ale_lb_get_state(ale_lb_t *h, double *pops, double *macros, double *t, int64_t *step)
{
    if (!h) return fail(ALE_LB_EINVAL, "null handle");
    int st = h->fp32 ? get_state_t(h, h->sf, h->sf.pop[h->cur], h->sf.mac[h->cur], pops, macros)
                     : get_state_t(h, h->sd, h->sd.pop[h->cur], h->sd.mac[h->cur], pops, macros);
    if (t) *t = h->t;
    if (step) *step = h->step;
    return st;
}

int ale_lb_set_state(ale_lb_t *h, const double *pops, const double *macros, double t, int64_t step)
{
    if (!h || !pops || !macros) return fail(ALE_LB_EINVAL, "null argument");
    int st = h->fp32 ? set_state_t(h, h->sf, pops, macros) : set_state_t(h, h->sd, pops, macros);
    h->t = t;
    h->step = step;
    return st;
}

int ale_lb_get_fields(ale_lb_t *h, double *rho, double *ux, double *uy, double *T, int32_t on_device)
{
    if (!h) return fail(ALE_LB_EINVAL, "null handle");
    const size_t N = h->N;
    double *dst[4] = {rho, ux, uy, T};
    if (on_device) {
        double *d = nullptr;
        HIP_OK(hipMalloc(&d, sizeof(double) * 4 * N));
        hipError_t e = h->fp32 ? launch_convert<float>(h->sf.mac[h->cur], d, N, 4, h->st)
                               : launch_convert<double>(h->sd.mac[h->cur], d, N, 4, h->st);
        HIP_OK(e);
        for (int c = 0; c < 4; ++c)
            if (dst[c]) HIP_OK(hipMemcpyAsync(dst[c], d + c * N, sizeof(double) * N, hipMemcpyDeviceToDevice, h->st));
        HIP_OK(hipStreamSynchronize(h->st));
        (void)hipFree(d);
        return ALE_LB_OK;
    }
    std::vector<double> mac(4 * N);
    int st = ale_lb_get_state(h, nullptr, mac.data(), nullptr, nullptr);
    if (st) return st;
    for (int c = 0; c < 4; ++c)
        if (dst[c]) std::memcpy(dst[c], mac.data() + c * N, sizeof(double) * N);
    return ALE_LB_OK;
}

int ale_lb_get_streamed(ale_lb_t *h, double *pops, int32_t *miss_wall, int32_t *miss_far)
{
    if (!h) return fail(ALE_LB_EINVAL, "null handle");
    int st = ALE_LB_OK;
    if (pops)
        st = h->fp32 ? get_state_t(h, h->sf, h->sf.ft, (const float *)nullptr, pops, nullptr)
                     : get_state_t(h, h->sd, h->sd.ft, (const double *)nullptr, pops, nullptr);
    if (st) return st;
    if (miss_wall || miss_far) {
        int *dm = h->fp32 ? h->sf.mask : h->sd.mask;
        if (!dm) return fail(ALE_LB_EINVAL, "missing masks need ALE_LB_F_KEEP_MASKS at create");
        std::vector<int> m(h->N);
        HIP_OK(hipMemcpyAsync(m.data(), dm, sizeof(int) * h->N, hipMemcpyDeviceToHost, h->st));
        HIP_OK(hipStreamSynchronize(h->st));
        for (int k = 0; k < h->N; ++k) {
            if (miss_wall) miss_wall[h->perm[k]] = m[k] & 0xffff;
            if (miss_far) miss_far[h->perm[k]] = (m[k] >> 16) & 0xffff;
        }
    }
    return ALE_LB_OK;
}

int ale_lb_get_correction(ale_lb_t *h, double *W, double *Xa)
{
    if (!h) return fail(ALE_LB_EINVAL, "null handle");
    const size_t N = h->N;
    std::vector<double> a(2 * N), b(2 * N);
    // two-component fields through the same converter (reads the first 2N entries)
    auto fetch2 = [&](auto *src, double *out) -> int {
        using R = std::remove_pointer_t<decltype(src)>;
        double *d = nullptr;
        HIP_OK(hipMalloc(&d, sizeof(double) * 2 * N));
        HIP_OK(launch_convert<R>(src, d, N, 2, h->st));
        std::vector<double> tmp(2 * N);
        HIP_OK(hipMemcpyAsync(tmp.data(), d, sizeof(double) * 2 * N, hipMemcpyDeviceToHost, h->st));
        HIP_OK(hipStreamSynchronize(h->st));
        (void)hipFree(d);
        for (int c = 0; c < 2; ++c)
            for (size_t k = 0; k < N; ++k) out[c * N + h->perm[k]] = tmp[c * N + k];
        return ALE_LB_OK;
    };
    int st = ALE_LB_OK;
    if (W) st = h->fp32 ? fetch2(h->sf.W, W) : fetch2(h->sd.W, W);
    if (!st && Xa) st = h->fp32 ? fetch2(h->sf.Xc, Xa) : fetch2(h->sd.Xc, Xa);
    return st;
}

int ale_lb_move_mesh(ale_lb_t *h, double t, double *x, double *Jinv, double *detJ, double *vg, int32_t on_device)
{
    if (!h) return fail(ALE_LB_EINVAL, "null handle");
    const size_t N = h->N;
    const MotionTime tf = motion_time(h->mo, t);
    int err = 0;
    HIP_OK(hipMemsetAsync(h->d_err, 0, sizeof(int), h->st));
    if (on_device) {
        HIP_OK(launch_move_mesh(h->dm, h->mo, tf, x, Jinv, detJ, vg, h->d_err, h->st));
    } else {
        double *d = nullptr;
        HIP_OK(hipMalloc(&d, sizeof(double) * 9 * N));
        HIP_OK(launch_move_mesh(h->dm, h->mo, tf, d, d + 2 * N, d + 6 * N, d + 7 * N, h->d_err, h->st));
        std::vector<double> tmp(9 * N);
        HIP_OK(hipMemcpyAsync(tmp.data(), d, sizeof(double) * 9 * N, hipMemcpyDeviceToHost, h->st));
        HIP_OK(hipStreamSynchronize(h->st));
        (void)hipFree(d);
        for (size_t k = 0; k < N; ++k) {
            const size_t a = h->perm[k];
            if (x) { x[2 * a] = tmp[2 * k]; x[2 * a + 1] = tmp[2 * k + 1]; }
            if (Jinv) for (int q = 0; q < 4; ++q) Jinv[4 * a + q] = tmp[2 * N + 4 * k + q];
            if (detJ) detJ[a] = tmp[6 * N + k];
            if (vg) { vg[2 * a] = tmp[7 * N + 2 * k]; vg[2 * a + 1] = tmp[7 * N + 2 * k + 1]; }
        }
    }
    HIP_OK(hipMemcpyAsync(&err, h->d_err, sizeof(int), hipMemcpyDeviceToHost, h->st));
    HIP_OK(hipStreamSynchronize(h->st));
    HIP_OK(hipMemsetAsync(h->d_err, 0, sizeof(int), h->st));
    HIP_OK(hipStreamSynchronize(h->st));
    if (err & ERR_JAC) return fail(ALE_LB_EJAC, "mapping Jacobian det <= 0 at t = %g", t);
    return ALE_LB_OK;
}

int ale_lb_forces(ale_lb_t *h, ale_lb_forces_t *out)
{
    if (!h || !out) return fail(ALE_LB_EINVAL, "null argument");
    const MotionTime tf = motion_time(h->mo, h->t);
    double F[6] = {0, 0, 0, 0, 0, 0};
    if (h->NWE > 0) {
        hipError_t e = h->fp32 ? launch_forces<float>(h->dm, h->sf.mac[h->cur], h->ph, h->mo, tf, h->d_part,
                                                      h->force_blocks, h->d_fout, h->st)
                               : launch_forces<double>(h->dm, h->sd.mac[h->cur], h->ph, h->mo, tf, h->d_part,
                                                       h->force_blocks, h->d_fout, h->st);
        HIP_OK(e);
        HIP_OK(hipMemcpyAsync(F, h->d_fout, sizeof(double) * 6, hipMemcpyDeviceToHost, h->st));
        HIP_OK(hipStreamSynchronize(h->st));
    }
    out->F_p[0] = F[0];
    out->F_p[1] = F[1];
    out->F_v[0] = F[2];
    out->F_v[1] = F[3];
    out->M_p = F[4];
    out->M_v = F[5];
    const double U2 = h->prm.u_inf[0] * h->prm.u_inf[0] + h->prm.u_inf[1] * h->prm.u_inf[1];
    const double qc = 0.5 * h->prm.rho_inf * U2 * h->prm.chord;
    out->cl = qc > 0 ? (F[1] + F[3]) / qc : 0.0;
    out->cd = qc > 0 ? (F[0] + F[2]) / qc : 0.0;
    out->cm = qc > 0 ? (F[4] + F[5]) / (qc * h->prm.chord) : 0.0;
    out->t = h->t;
    return ALE_LB_OK;
}

int ale_lb_info(ale_lb_t *h, int64_t *out, int32_t n)
{
    if (!h || !out) return fail(ALE_LB_EINVAL, "null argument");
    const int64_t v[6] = {h->N, h->E, h->NWE, h->NW, int64_t(h->dev_bytes), h->fp32 ? 4 : 8};
    for (int k = 0; k < n && k < 6; ++k) out[k] = v[k];
    return ALE_LB_OK;
}

int ale_lb_node_order(ale_lb_t *h, int32_t *perm)
{
    if (!h || !perm) return fail(ALE_LB_EINVAL, "null argument");
    std::memcpy(perm, h->perm.data(), sizeof(int) * h->N);
    return ALE_LB_OK;
}

}  // extern "C"
