/* A plain C caller of the library's C-ABI (include/alelb.h), with no Python,
 * PyTorch or HIP code of its own: it shows that the boundary stands alone.
 *
 *   c_abi_check <input> <output>
 *
 * <input> (native byte order), written by tests/test_gpu_c_abi.py:
 *   int32  magic 0x424c4541, n_nodes, n_elems, nodes_per_elem, n_wall_edges,
 *          steps, sizeof(ale_lb_params_t) as the writer laid it out
 *   double period[2], gamma, Pr
 *   double X[2 n_nodes]; int32 elem[nodes_per_elem n_elems];
 *   int32 nbr[nf n_elems]; int8 pshift[nf n_elems]   (nf = 3 or 4 edges)
 *   int32 wall_edges[2 n_wall_edges]
 *   bytes ale_lb_params_t (stream NULL)
 *   double rho[n], ux[n], uy[n], T[n]
 * <output>:
 *   double fields[4 n] (rho, ux, uy, T), pops[18 n], macros[4 n], t;
 *   int64 step; ale_lb_forces_t (when the mesh has walls)
 *
 * Exit status 0 on success; otherwise the library's error is printed. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "alelb.h"

static FILE *fin;

static void get(void *p, size_t n)
{
    if (n && fread(p, 1, n, fin) != n) {
        fprintf(stderr, "c_abi_check: short input\n");
        exit(2);
    }
}

static void *take(size_t n)
{
    void *p = malloc(n ? n : 1);
    if (!p) {
        fprintf(stderr, "c_abi_check: out of host memory\n");
        exit(2);
    }
    get(p, n);
    return p;
}

static int check(int code, const char *what)
{
    if (code != ALE_LB_OK) fprintf(stderr, "c_abi_check: %s: %d %s\n", what, code, ale_lb_last_error());
    return code;
}

int main(int argc, char **argv)
{
    if (argc != 3) {
        fprintf(stderr, "usage: c_abi_check <input> <output>\n");
        return 2;
    }
    fin = fopen(argv[1], "rb");
    if (!fin) {
        perror(argv[1]);
        return 2;
    }
    int32_t hdr[7];
    get(hdr, sizeof hdr);
    if (hdr[0] != 0x424c4541) {
        fprintf(stderr, "c_abi_check: bad magic\n");
        return 2;
    }
    const int32_t N = hdr[1], E = hdr[2], nv = hdr[3], nwe = hdr[4], steps = hdr[5];
    if (hdr[6] != (int32_t)sizeof(ale_lb_params_t)) {
        fprintf(stderr, "c_abi_check: params are %d bytes in the input, %zu in alelb.h\n", hdr[6],
                sizeof(ale_lb_params_t));
        return 3;
    }
    const int nf = nv == 9 ? 4 : 3;
    double d4[4];
    get(d4, sizeof d4);
    ale_lb_mesh_t mesh;
    memset(&mesh, 0, sizeof mesh);
    mesh.n_nodes = N;
    mesh.n_elems = E;
    mesh.nodes_per_elem = nv;
    mesh.period[0] = d4[0];
    mesh.period[1] = d4[1];
    mesh.X = take(sizeof(double) * 2 * (size_t)N);
    mesh.elem = take(sizeof(int32_t) * (size_t)nv * E);
    mesh.nbr = take(sizeof(int32_t) * (size_t)nf * E);
    mesh.pshift = take((size_t)nf * E);
    mesh.n_wall_edges = nwe;
    mesh.wall_edges = take(sizeof(int32_t) * 2 * (size_t)nwe);
    ale_lb_params_t params;
    get(&params, sizeof params);
    params.stream = NULL;
    ale_lb_lattice_t lattice;
    memset(&lattice, 0, sizeof lattice);
    lattice.Q = 9;
    lattice.gamma = d4[2];
    lattice.Pr = d4[3];
    double *init = take(sizeof(double) * 4 * (size_t)N);
    fclose(fin);

    ale_lb_t *h = NULL;
    if (check(ale_lb_create(&mesh, &lattice, &params, &h), "create")) return 1;
    double *fields = malloc(sizeof(double) * 4 * (size_t)N), *pops = malloc(sizeof(double) * 18 * (size_t)N);
    double *macros = malloc(sizeof(double) * 4 * (size_t)N);
    double t = 0.0;
    int64_t step = 0;
    ale_lb_forces_t forces;
    memset(&forces, 0, sizeof forces);
    int st = check(ale_lb_init_fields(h, init, init + N, init + 2 * (size_t)N, init + 3 * (size_t)N), "init_fields");
    if (!st) st = check(ale_lb_step(h, steps), "step");
    if (!st)
        st = check(ale_lb_get_fields(h, fields, fields + N, fields + 2 * (size_t)N, fields + 3 * (size_t)N, 0),
                   "get_fields");
    if (!st) st = check(ale_lb_get_state(h, pops, macros, &t, &step), "get_state");
    if (!st && nwe > 0) st = check(ale_lb_forces(h, &forces), "forces");
    ale_lb_destroy(h);
    if (st) return 1;

    FILE *fo = fopen(argv[2], "wb");
    if (!fo) {
        perror(argv[2]);
        return 2;
    }
    fwrite(fields, sizeof(double), 4 * (size_t)N, fo);
    fwrite(pops, sizeof(double), 18 * (size_t)N, fo);
    fwrite(macros, sizeof(double), 4 * (size_t)N, fo);
    fwrite(&t, sizeof t, 1, fo);
    fwrite(&step, sizeof step, 1, fo);
    if (nwe > 0) fwrite(&forces, sizeof forces, 1, fo);
    fclose(fo);
    printf("c_abi_check: %d nodes, %d steps done\n", N, steps);
    return 0;
}
