/* Test driver (CPU): runs the FP64 oracle's models on a mesh read from a
 * binary file, for the address/undefined-behaviour sanitizer build of the
 * oracle.  File layout: int32 N, E, V; float64 radius; then the arrays of
 * or_mesh_in in declaration order (int32 index arrays, float64 geometry);
 * then float64 state arrays (ps[N], Theta[N][K], u[E][K], w[N][K+1],
 * phi[N][K+1], tracer F[E][K], dpi[N][K], q[N][K][T], vflux[N][K+1]). */
#include <stdio.h>
#include <stdlib.h>

#include "oracle.h"

static void *rd(FILE *f, size_t n, size_t sz)
{
    void *p = malloc(n * sz ? n * sz : 1);
    if (fread(p, sz, n, f) != n) { fprintf(stderr, "short read\n"); exit(2); }
    return p;
}

int main(int argc, char **argv)
{
    if (argc < 4) return 2;
    FILE *f = fopen(argv[1], "rb");
    const int K = atoi(argv[2]), T = atoi(argv[3]);
    int hdr[3];
    double radius;
    if (!f || fread(hdr, 4, 3, f) != 3 || fread(&radius, 8, 1, f) != 1) return 2;
    const int N = hdr[0], E = hdr[1], V = hdr[2];
    or_mesh_in in;
    in.N = N; in.E = E; in.V = V;
    in.cells_on_edge = rd(f, 2 * (size_t)E, 4);
    in.vertices_on_edge = rd(f, 2 * (size_t)E, 4);
    in.eoc_offset = rd(f, (size_t)N + 1, 4);
    in.edges_on_cell = rd(f, 2 * (size_t)E, 4);
    in.vertices_on_cell = rd(f, 2 * (size_t)E, 4);
    in.cells_on_vertex = rd(f, 3 * (size_t)V, 4);
    in.edges_on_vertex = rd(f, 3 * (size_t)V, 4);
    in.xCell = rd(f, 3 * (size_t)N, 8);
    in.xVertex = rd(f, 3 * (size_t)V, 8);
    in.xEdge = rd(f, 3 * (size_t)E, 8);
    in.dEdge = rd(f, (size_t)E, 8);
    in.lEdge = rd(f, (size_t)E, 8);
    in.areaCell = rd(f, (size_t)N, 8);
    in.areaVertex = rd(f, (size_t)V, 8);
    in.kiteArea = rd(f, 3 * (size_t)V, 8);
    in.fVertex = rd(f, (size_t)V, 8);
    in.radius = radius;
    double *ps = rd(f, N, 8), *Th = rd(f, (size_t)N * K, 8), *u = rd(f, (size_t)E * K, 8);
    double *w = rd(f, (size_t)N * (K + 1), 8), *phi = rd(f, (size_t)N * (K + 1), 8);
    double *F = rd(f, (size_t)E * K, 8), *dpi = rd(f, (size_t)N * K, 8), *q = rd(f, (size_t)N * K * T, 8);
    double *vf = rd(f, (size_t)N * (K + 1), 8);
    fclose(f);
    double *sig = malloc(sizeof(double) * (K + 1));
    for (int k = 0; k <= K; k++) sig[k] = (double)k / K;
    or_params p = {K, T, 60.0, 9.80616, 287.0, 1004.5, 1.0e5, 1000.0, sig, 1, NULL};
    or_mesh *m = or_mesh_build(&in);
    if (!m) return 3;
    double *Fa = calloc((size_t)E * K, 8), *Ma = calloc((size_t)N * (K + 1), 8);
    double *ps2 = malloc(sizeof(double) * N), *Th2 = malloc(sizeof(double) * N * K), *u2 = malloc(sizeof(double) * E * K);
    for (int i = 0; i < N; i++) ps2[i] = ps[i];
    for (long x = 0; x < (long)N * K; x++) Th2[x] = Th[x];
    for (long x = 0; x < (long)E * K; x++) u2[x] = u[x];
    or_hdc_run_flux(m, &p, ps2, Th2, u2, 2, Fa, Ma);
    or_ndc_run(m, &p, ps, Th, u, w, phi, 1);
    p.dt = 600.0;
    or_tracer_run(m, &p, F, vf, dpi, q, 1);
    double *h = malloc(sizeof(double) * N), *b = calloc(N, 8), *u1 = malloc(sizeof(double) * E);
    for (int i = 0; i < N; i++) h[i] = 1000.0;
    for (int e = 0; e < E; e++) u1[e] = 1.0;
    p.K = 1;
    or_sw_run(m, &p, h, u1, b, 1);
    or_mesh_free(m);
    void *own[] = {(void *)in.cells_on_edge, (void *)in.vertices_on_edge, (void *)in.eoc_offset,
                   (void *)in.edges_on_cell, (void *)in.vertices_on_cell, (void *)in.cells_on_vertex,
                   (void *)in.edges_on_vertex, (void *)in.xCell, (void *)in.xVertex, (void *)in.xEdge,
                   (void *)in.dEdge, (void *)in.lEdge, (void *)in.areaCell, (void *)in.areaVertex,
                   (void *)in.kiteArea, (void *)in.fVertex, ps, Th, u, w, phi, F, dpi, q, vf, sig, Fa, Ma,
                   ps2, Th2, u2, h, b, u1};
    for (size_t j = 0; j < sizeof(own) / sizeof(own[0]); j++) free(own[j]);
    printf("ok\n");
    return 0;
}
