/*
 * FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Plain loops, double precision everywhere, each output written by one
 * thread in a fixed order (OpenMP over entities only).  Built with
 * -O2 -ffp-contract=off so that no fused multiply-add changes the rounding.
 *
 * Paper anchors (arXiv 2404.08849): C-grid staggering and RK / forward-
 * backward / HEVI integrators (Section 2.1); continuity, theta_m, momentum,
 * w, phi, hydrostatic, state and tracer equations (Section 2.3, Eqs. 3-10);
 * third-order upwind flux with an FCT limiter (Section 2.1); error norms
 * L1/L2/Linf (Section 2.2, Eqs. 1-2).  Discrete operators follow the TRiSK
 * reading stated in oracle.h.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXDEG 6

struct or_mesh {
    or_mesh_in m;
    int *coc;          /* [2E] neighbour across CSR slot                    */
    double *sgn;       /* [2E] s_{e,i} = +1 if i == c1(e) else -1            */
    double *sgnv;      /* [3V] s'_{e,v} = +1 if v == v2(e) else -1           */
    int *slot;         /* [E][2] CSR slot of e in c1 and in c2               */
    int *tk_off;       /* [E+1] TRiSK list offsets                           */
    int *tk_e;         /* TRiSK edges e'                                     */
    double *tk_w;      /* TRiSK weights w_{e,e'}                             */
    double *hw;        /* [2E][MAXDEG] directional second-derivative weights */
};

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------ */
/* small vector helpers                                                */
/* ------------------------------------------------------------------ */
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
static double norm3(const double *a) { return sqrt(dot3(a, a)); }
static double arc3(const double *a, const double *b)
{
    double c[3];
    cross3(a, b, c);
    return atan2(norm3(c), dot3(a, b));
}

/* Gaussian elimination with partial pivoting: solve A X = B, A n x n, B n x m
 * (row-major, overwritten).  Returns 0 on success. */
static int gauss_solve(int n, int m, double *A, double *B)
{
    for (int c = 0; c < n; c++) {
        int p = c;
        for (int r = c + 1; r < n; r++)
            if (fabs(A[r * n + c]) > fabs(A[p * n + c])) p = r;
        if (A[p * n + c] == 0.0) return -1;
        if (p != c) {
            for (int j = 0; j < n; j++) { double t = A[c * n + j]; A[c * n + j] = A[p * n + j]; A[p * n + j] = t; }
            for (int j = 0; j < m; j++) { double t = B[c * m + j]; B[c * m + j] = B[p * m + j]; B[p * m + j] = t; }
        }
        for (int r = c + 1; r < n; r++) {
            double f = A[r * n + c] / A[c * n + c];
            for (int j = c; j < n; j++) A[r * n + j] -= f * A[c * n + j];
            for (int j = 0; j < m; j++) B[r * m + j] -= f * B[c * m + j];
        }
    }
    for (int c = n - 1; c >= 0; c--) {
        for (int j = 0; j < m; j++) {
            double s = B[c * m + j];
            for (int k = c + 1; k < n; k++) s -= A[c * n + k] * B[k * m + j];
            B[c * m + j] = s / A[c * n + c];
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* mesh tables                                                         */
/* ------------------------------------------------------------------ */
static double kite_of(const or_mesh_in *m, int v, int cell)
{
    for (int j = 0; j < 3; j++)
        if (m->cells_on_vertex[3 * v + j] == cell) return m->kiteArea[3 * v + j];
    return NAN;
}

void or_mesh_free(or_mesh *h)
{
    if (!h) return;
    free(h->coc); free(h->sgn); free(h->sgnv); free(h->slot);
    free(h->tk_off); free(h->tk_e); free(h->tk_w); free(h->hw);
    free(h);
}

/*
 * Tables derived from the mesh:
 *  - s_{e,i} (outward sign of n_e for cell i) and s'_{e,v} (sign of n_e in the
 *    counter-clockwise circulation around v);
 *  - TRiSK tangential-flux weights: for edge e and each cell i of e, walk i's
 *    edges counter-clockwise from e (e_0 = e, e_1 .. e_{n-1}); v_k is the vertex
 *    between e_{k-1} and e_k and S_j = sum_{k<=j} R_{i,v_k} / A_i; then
 *    w_{e,e_j} = s_{e,i} s_{e_j,i} (1/2 - S_j).  With these weights
 *    (1/d_e) sum w l F reconstructs the tangential flux of a streamfunction
 *    field exactly as the gradient of its kite-averaged cell values;
 *  - directional second-derivative weights from an unweighted least-squares
 *    quadratic fit q_k - q_i = a x + b y + c x^2 + d xy + e y^2 over the
 *    cell's neighbours, in azimuthal-equidistant coordinates (arc length,
 *    bearing) with the first axis towards the first listed neighbour:
 *    q''_{i,e_j} = sum_k W[i][j][k] (q_{nb_k} - q_i) is the second derivative
 *    along the direction of neighbour j.
 */
or_mesh *or_mesh_build(const or_mesh_in *in)
{
    const int N = in->N, E = in->E, V = in->V;
    or_mesh *h = (or_mesh *)calloc(1, sizeof(or_mesh));
    h->m = *in;
    const int *off = in->eoc_offset;
    for (int i = 0; i < N; i++) {
        int n = off[i + 1] - off[i];
        if (n < 3 || n > MAXDEG) { or_mesh_free(h); return NULL; }
    }
    h->coc = (int *)malloc(sizeof(int) * 2 * E);
    h->sgn = (double *)malloc(sizeof(double) * 2 * E);
    h->sgnv = (double *)malloc(sizeof(double) * 3 * V);
    h->slot = (int *)malloc(sizeof(int) * 2 * E);
    for (int i = 0; i < N; i++) {
        for (int j = off[i]; j < off[i + 1]; j++) {
            int e = in->edges_on_cell[j];
            int c1 = in->cells_on_edge[2 * e], c2 = in->cells_on_edge[2 * e + 1];
            h->coc[j] = (c1 == i) ? c2 : c1;
            h->sgn[j] = (c1 == i) ? 1.0 : -1.0;
            h->slot[2 * e + ((c1 == i) ? 0 : 1)] = j - off[i];
        }
    }
    for (int v = 0; v < V; v++)
        for (int j = 0; j < 3; j++) {
            int e = in->edges_on_vertex[3 * v + j];
            h->sgnv[3 * v + j] = (in->vertices_on_edge[2 * e + 1] == v) ? 1.0 : -1.0;
        }

    /* TRiSK */
    h->tk_off = (int *)malloc(sizeof(int) * (E + 1));
    h->tk_off[0] = 0;
    for (int e = 0; e < E; e++) {
        int c1 = in->cells_on_edge[2 * e], c2 = in->cells_on_edge[2 * e + 1];
        h->tk_off[e + 1] = h->tk_off[e] + (off[c1 + 1] - off[c1] - 1) + (off[c2 + 1] - off[c2] - 1);
    }
    h->tk_e = (int *)malloc(sizeof(int) * h->tk_off[E]);
    h->tk_w = (double *)malloc(sizeof(double) * h->tk_off[E]);
    for (int e = 0; e < E; e++) {
        int pos = h->tk_off[e];
        for (int side = 0; side < 2; side++) {
            int i = in->cells_on_edge[2 * e + side];
            int n = off[i + 1] - off[i];
            int j0 = h->slot[2 * e + side];
            double s_ei = h->sgn[off[i] + j0];
            double S = 0.0;
            for (int step = 1; step < n; step++) {
                int j = (j0 + step) % n;
                int vk = in->vertices_on_cell[off[i] + j];
                S += kite_of(in, vk, i) / in->areaCell[i];
                h->tk_e[pos] = in->edges_on_cell[off[i] + j];
                h->tk_w[pos] = s_ei * h->sgn[off[i] + j] * (0.5 - S);
                pos++;
            }
        }
    }

    /* Hessian (directional second derivative) weights */
    h->hw = (double *)calloc((size_t)2 * E * MAXDEG, sizeof(double));
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (int i = 0; i < N; i++) {
        const int n = off[i + 1] - off[i];
        const double *xi = in->xCell + 3 * i;
        double e1[3], e2[3], X[MAXDEG], Y[MAXDEG], cb[MAXDEG], sb[MAXDEG];
        const double *x0 = in->xCell + 3 * h->coc[off[i]];
        double d0 = dot3(x0, xi);
        for (int c = 0; c < 3; c++) e1[c] = x0[c] - d0 * xi[c];
        double ne1 = norm3(e1);
        for (int c = 0; c < 3; c++) e1[c] /= ne1;
        cross3(xi, e1, e2);
        double s = 0.0;
        for (int k = 0; k < n; k++) {
            const double *xk = in->xCell + 3 * h->coc[off[i] + k];
            double r = arc3(xi, xk);
            double dk = dot3(xk, xi), t[3];
            for (int c = 0; c < 3; c++) t[c] = xk[c] - dk * xi[c];
            double tn = norm3(t);
            cb[k] = dot3(t, e1) / tn;
            sb[k] = dot3(t, e2) / tn;
            X[k] = r * cb[k];
            Y[k] = r * sb[k];
            s += r;
        }
        s /= n;
        /* normal equations of the scaled fit: (M^T M) P = M^T, M rows [x, y, x^2, xy, y^2] */
        double Mr[MAXDEG][5], A[25], B[5 * MAXDEG];
        for (int k = 0; k < n; k++) {
            double xs = X[k] / s, ys = Y[k] / s;
            Mr[k][0] = xs; Mr[k][1] = ys; Mr[k][2] = xs * xs; Mr[k][3] = xs * ys; Mr[k][4] = ys * ys;
        }
        for (int r = 0; r < 5; r++) {
            for (int c = 0; c < 5; c++) {
                double acc = 0.0;
                for (int k = 0; k < n; k++) acc += Mr[k][r] * Mr[k][c];
                A[r * 5 + c] = acc;
            }
            for (int k = 0; k < n; k++) B[r * n + k] = Mr[k][r];
        }
        if (gauss_solve(5, n, A, B)) { bad += 1; continue; }
        double L = in->radius * s;
        double inv = 1.0 / (L * L);
        for (int j = 0; j < n; j++)
            for (int k = 0; k < n; k++)
                h->hw[(size_t)(off[i] + j) * MAXDEG + k] =
                    (2.0 * B[2 * n + k] * cb[j] * cb[j] + 2.0 * B[3 * n + k] * cb[j] * sb[j] +
                     2.0 * B[4 * n + k] * sb[j] * sb[j]) * inv;
    }
    if (bad) { or_mesh_free(h); return NULL; }
    return h;
}

int or_table_sizes(const or_mesh *h, int *n_trisk)
{
    *n_trisk = h->tk_off[h->m.E];
    return 0;
}
void or_get_cells_on_cell(const or_mesh *h, int *out) { memcpy(out, h->coc, sizeof(int) * 2 * h->m.E); }
void or_get_edge_sign(const or_mesh *h, double *out) { memcpy(out, h->sgn, sizeof(double) * 2 * h->m.E); }
void or_get_vertex_sign(const or_mesh *h, double *out) { memcpy(out, h->sgnv, sizeof(double) * 3 * h->m.V); }
void or_get_trisk(const or_mesh *h, int *off, int *edge, double *w)
{
    memcpy(off, h->tk_off, sizeof(int) * (h->m.E + 1));
    memcpy(edge, h->tk_e, sizeof(int) * h->tk_off[h->m.E]);
    memcpy(w, h->tk_w, sizeof(double) * h->tk_off[h->m.E]);
}
void or_get_hessian(const or_mesh *h, double *w) { memcpy(w, h->hw, sizeof(double) * 2 * h->m.E * MAXDEG); }

/* ------------------------------------------------------------------ */
/* operators (K layers, level innermost)                               */
/* ------------------------------------------------------------------ */

/* G_e psi = (psi_c2 - psi_c1) / d_e */
void or_gradient(const or_mesh *h, int K, const double *psi, double *out)
{
    const or_mesh_in *m = &h->m;
#pragma omp parallel for schedule(static)
    for (int e = 0; e < m->E; e++) {
        int c1 = m->cells_on_edge[2 * e], c2 = m->cells_on_edge[2 * e + 1];
        for (int k = 0; k < K; k++)
            out[(size_t)e * K + k] = (psi[(size_t)c2 * K + k] - psi[(size_t)c1 * K + k]) / m->dEdge[e];
    }
}

/* D_i F = (1/A_i) sum_{e in EC(i)} s_{e,i} l_e F_e, summed in CSR order */
void or_divergence(const or_mesh *h, int K, const double *F, double *out)
{
    const or_mesh_in *m = &h->m;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < m->N; i++) {
        for (int k = 0; k < K; k++) {
            double acc = 0.0;
            for (int j = m->eoc_offset[i]; j < m->eoc_offset[i + 1]; j++) {
                int e = m->edges_on_cell[j];
                acc += h->sgn[j] * m->lEdge[e] * F[(size_t)e * K + k];
            }
            out[(size_t)i * K + k] = acc / m->areaCell[i];
        }
    }
}

/* zeta_v = (1/A_v) sum_{e in EV(v)} s'_{e,v} d_e u_e */
void or_curl(const or_mesh *h, int K, const double *u, double *out)
{
    const or_mesh_in *m = &h->m;
#pragma omp parallel for schedule(static)
    for (int v = 0; v < m->V; v++) {
        for (int k = 0; k < K; k++) {
            double acc = 0.0;
            for (int j = 0; j < 3; j++) {
                int e = m->edges_on_vertex[3 * v + j];
                acc += h->sgnv[3 * v + j] * m->dEdge[e] * u[(size_t)e * K + k];
            }
            out[(size_t)v * K + k] = acc / m->areaVertex[v];
        }
    }
}

/* K_i = (1/A_i) sum_{e in EC(i)} (l_e d_e / 4) u_e^2 */
void or_kinetic_energy(const or_mesh *h, int K, const double *u, double *out)
{
    const or_mesh_in *m = &h->m;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < m->N; i++) {
        for (int k = 0; k < K; k++) {
            double acc = 0.0;
            for (int j = m->eoc_offset[i]; j < m->eoc_offset[i + 1]; j++) {
                int e = m->edges_on_cell[j];
                double ue = u[(size_t)e * K + k];
                acc += 0.25 * m->lEdge[e] * m->dEdge[e] * ue * ue;
            }
            out[(size_t)i * K + k] = acc / m->areaCell[i];
        }
    }
}

/* h_v = (1/A_v) sum_i R_{i,v} h_i */
void or_vertex_mass(const or_mesh *h, int K, const double *hc, double *out)
{
    const or_mesh_in *m = &h->m;
#pragma omp parallel for schedule(static)
    for (int v = 0; v < m->V; v++) {
        for (int k = 0; k < K; k++) {
            double acc = 0.0;
            for (int j = 0; j < 3; j++)
                acc += m->kiteArea[3 * v + j] * hc[(size_t)m->cells_on_vertex[3 * v + j] * K + k];
            out[(size_t)v * K + k] = acc / m->areaVertex[v];
        }
    }
}

/* F_perp_e = (1/d_e) sum_{e'} w_{e,e'} l_{e'} F_{e'} */
void or_perp_flux(const or_mesh *h, int K, const double *F, double *out)
{
    const or_mesh_in *m = &h->m;
#pragma omp parallel for schedule(static)
    for (int e = 0; e < m->E; e++) {
        for (int k = 0; k < K; k++) {
            double acc = 0.0;
            for (int t = h->tk_off[e]; t < h->tk_off[e + 1]; t++) {
                int ep = h->tk_e[t];
                acc += h->tk_w[t] * m->lEdge[ep] * F[(size_t)ep * K + k];
            }
            out[(size_t)e * K + k] = acc / m->dEdge[e];
        }
    }
}

/* Q_e = (1/d_e) sum_{e'} w_{e,e'} l_{e'} F_{e'} (q_e + q_{e'})/2, q_e = (q_v1 + q_v2)/2 */
void or_coriolis(const or_mesh *h, int K, const double *F, const double *qv, double *out)
{
    const or_mesh_in *m = &h->m;
#pragma omp parallel for schedule(static)
    for (int e = 0; e < m->E; e++) {
        for (int k = 0; k < K; k++) {
            double qe = 0.5 * (qv[(size_t)m->vertices_on_edge[2 * e] * K + k] +
                               qv[(size_t)m->vertices_on_edge[2 * e + 1] * K + k]);
            double acc = 0.0;
            for (int t = h->tk_off[e]; t < h->tk_off[e + 1]; t++) {
                int ep = h->tk_e[t];
                double qep = 0.5 * (qv[(size_t)m->vertices_on_edge[2 * ep] * K + k] +
                                    qv[(size_t)m->vertices_on_edge[2 * ep + 1] * K + k]);
                acc += h->tk_w[t] * m->lEdge[ep] * F[(size_t)ep * K + k] * 0.5 * (qe + qep);
            }
            out[(size_t)e * K + k] = acc / m->dEdge[e];
        }
    }
}

/* q''_{i,e_j} = sum_k W[i][j][k] (q_{nb_k} - q_i), one value per CSR slot and level */
void or_hessian_dir(const or_mesh *h, int K, const double *q, double *out)
{
    const or_mesh_in *m = &h->m;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < m->N; i++) {
        int o = m->eoc_offset[i], n = m->eoc_offset[i + 1] - o;
        for (int j = 0; j < n; j++)
            for (int k = 0; k < K; k++) {
                double acc = 0.0;
                for (int r = 0; r < n; r++)
                    acc += h->hw[(size_t)(o + j) * MAXDEG + r] * (q[(size_t)h->coc[o + r] * K + k] - q[(size_t)i * K + k]);
                out[(size_t)(o + j) * K + k] = acc;
            }
    }
}

/* Third-order upwind edge value (Skamarock & Gassmann 2011 flux form, beta = 1):
 * qe = (q1 + q2)/2 - d^2/12 (q''1 + q''2) + sgn(F) d^2/12 (q''2 - q''1), sgn(0) = +1. */
static double edge_value3(double q1, double q2, double h1, double h2, double d, double F)
{
    double c = d * d / 12.0;
    double sg = (F >= 0.0) ? 1.0 : -1.0;
    return 0.5 * (q1 + q2) - c * (h1 + h2) + sg * c * (h2 - h1);
}

void or_edge_value3_formula(int n, const double *qc1, const double *qc2, const double *h1,
                            const double *h2, const double *d, const double *F, double *out)
{
    for (int i = 0; i < n; i++) out[i] = edge_value3(qc1[i], qc2[i], h1[i], h2[i], d[i], F[i]);
}

/* q~_e for every edge and level from cell values q [N][K] and the sign of F [E][K] */
void or_edge_value3(const or_mesh *h, int K, const double *q, const double *F, double *out)
{
    const or_mesh_in *m = &h->m;
    double *hd = (double *)malloc(sizeof(double) * 2 * m->E * K);
    or_hessian_dir(h, K, q, hd);
#pragma omp parallel for schedule(static)
    for (int e = 0; e < m->E; e++) {
        int c1 = m->cells_on_edge[2 * e], c2 = m->cells_on_edge[2 * e + 1];
        size_t s1 = (size_t)m->eoc_offset[c1] + h->slot[2 * e];
        size_t s2 = (size_t)m->eoc_offset[c2] + h->slot[2 * e + 1];
        for (int k = 0; k < K; k++)
            out[(size_t)e * K + k] = edge_value3(q[(size_t)c1 * K + k], q[(size_t)c2 * K + k],
                                                 hd[s1 * K + k], hd[s2 * K + k], m->dEdge[e],
                                                 F[(size_t)e * K + k]);
    }
    free(hd);
}

/* Thomas algorithm for a tridiagonal system (no pivoting): sub[0] and sup[n-1] unused. */
int or_thomas(int n, const double *sub, const double *diag, const double *sup, const double *rhs, double *x)
{
    double *cp = (double *)malloc(sizeof(double) * n);
    double *dp = (double *)malloc(sizeof(double) * n);
    double den = diag[0];
    if (den == 0.0) { free(cp); free(dp); return -1; }
    cp[0] = sup[0] / den;
    dp[0] = rhs[0] / den;
    for (int i = 1; i < n; i++) {
        den = diag[i] - sub[i] * cp[i - 1];
        if (den == 0.0) { free(cp); free(dp); return -1; }
        cp[i] = (i < n - 1) ? sup[i] / den : 0.0;
        dp[i] = (rhs[i] - sub[i] * dp[i - 1]) / den;
    }
    x[n - 1] = dp[n - 1];
    for (int i = n - 2; i >= 0; i--) x[i] = dp[i] - cp[i] * x[i + 1];
    free(cp); free(dp);
    return 0;
}

static double *dalloc(size_t n) { return (double *)malloc(sizeof(double) * (n ? n : 1)); }

static const double RK3_FRAC[3] = {1.0 / 3.0, 0.5, 1.0};

/* ------------------------------------------------------------------ */
/* shallow water: h at cells, u at edges (single layer)                */
/* ------------------------------------------------------------------ */
/*
 * dh/dt = -D(F), F_e = (h_c1 + h_c2)/2 u_e
 * du/dt = Q_e - G_e K - g G_e (h + b)
 * Wicker-Skamarock RK3 (dt/3, dt/2, dt from the step's start state); in each
 * stage h is updated first and the gravity term uses the updated h
 * (forward-backward), or the stage's input h when p->no_fb is set.
 */
void or_sw_run(const or_mesh *h, const or_params *p, double *hs, double *us, const double *b, int nsteps)
{
    const or_mesh_in *m = &h->m;
    const int N = m->N, E = m->E, V = m->V;
    double *h0 = dalloc(N), *u0 = dalloc(E), *F = dalloc(E), *div = dalloc(N), *ke = dalloc(N);
    double *zeta = dalloc(V), *hv = dalloc(V), *qv = dalloc(V), *Q = dalloc(E), *hn = dalloc(N);
    for (int step = 0; step < nsteps; step++) {
        memcpy(h0, hs, sizeof(double) * N);
        memcpy(u0, us, sizeof(double) * E);
        for (int s = 0; s < 3; s++) {
            double dts = RK3_FRAC[s] * p->dt;
            for (int e = 0; e < E; e++)
                F[e] = 0.5 * (hs[m->cells_on_edge[2 * e]] + hs[m->cells_on_edge[2 * e + 1]]) * us[e];
            or_divergence(h, 1, F, div);
            or_kinetic_energy(h, 1, us, ke);
            or_curl(h, 1, us, zeta);
            or_vertex_mass(h, 1, hs, hv);
            for (int v = 0; v < V; v++) qv[v] = (zeta[v] + m->fVertex[v]) / hv[v];
            or_coriolis(h, 1, F, qv, Q);
            for (int i = 0; i < N; i++) hn[i] = h0[i] + dts * (-div[i]);
            for (int e = 0; e < E; e++) {
                int c1 = m->cells_on_edge[2 * e], c2 = m->cells_on_edge[2 * e + 1];
                double gk = (ke[c2] - ke[c1]) / m->dEdge[e];
                const double *hg = p->no_fb ? hs : hn;
                double gh = p->grav * ((hg[c2] + b[c2]) - (hg[c1] + b[c1])) / m->dEdge[e];
                us[e] = u0[e] + dts * (Q[e] - gk - gh);
            }
            memcpy(hs, hn, sizeof(double) * N);
        }
    }
    free(h0); free(u0); free(F); free(div); free(ke); free(zeta); free(hv); free(qv); free(Q); free(hn);
}

/* ------------------------------------------------------------------ */
/* shared pieces of the 3-D dry dynamical core                         */
/* ------------------------------------------------------------------ */

/* layer mass delta pi_k = (sigma_{k+1} - sigma_k)(pi_s - pi_t) */
static void layer_mass(const or_params *p, int N, const double *ps, double *dpi)
{
    const int K = p->K;
    for (int i = 0; i < N; i++)
        for (int k = 0; k < K; k++)
            dpi[(size_t)i * K + k] = (p->sigma[k + 1] - p->sigma[k]) * (ps[i] - p->ptop);
}

/* normal mass flux F_{e,k} = (dpi_c1 + dpi_c2)/2 u_{e,k} */
static void mass_flux(const or_mesh_in *m, int K, const double *dpi, const double *u, double *F)
{
#pragma omp parallel for schedule(static)
    for (int e = 0; e < m->E; e++) {
        int c1 = m->cells_on_edge[2 * e], c2 = m->cells_on_edge[2 * e + 1];
        for (int k = 0; k < K; k++)
            F[(size_t)e * K + k] = 0.5 * (dpi[(size_t)c1 * K + k] + dpi[(size_t)c2 * K + k]) * u[(size_t)e * K + k];
    }
}

/* dpi_s/dt = -sum_k D_k; vertical mass flux through interface k (positive
 * towards the surface): mdot_k = -sum_{j<k} D_j - sigma_k dpi_s/dt, zero at
 * the top and bottom. */
static void column_mass(const or_params *p, int N, const double *D, double *dps, double *mdot)
{
    const int K = p->K;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < N; i++) {
        double s = 0.0;
        for (int k = 0; k < K; k++) s += D[(size_t)i * K + k];
        dps[i] = -s;
        double acc = 0.0;
        mdot[(size_t)i * (K + 1)] = 0.0;
        for (int k = 0; k < K; k++) {
            acc += D[(size_t)i * K + k];
            mdot[(size_t)i * (K + 1) + k + 1] = (k == K - 1) ? 0.0 : -acc - p->sigma[k + 1] * dps[i];
        }
    }
}

/* theta_m transport tendency: -D(F theta~) - (mdot_{k+1} theta_{k+1/2} - mdot_k theta_{k-1/2}),
 * theta~ the third-order upwind edge value, theta at an interface the mean of the two layers. */
static void theta_tendency(const or_mesh *h, const or_params *p, const double *F, const double *theta,
                           const double *mdot, double *tend, double *work_e, double *work_c)
{
    const or_mesh_in *m = &h->m;
    const int K = p->K;
    or_edge_value3(h, K, theta, F, work_e);
    for (size_t x = 0; x < (size_t)m->E * K; x++) work_e[x] *= F[x];
    or_divergence(h, K, work_e, work_c);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < m->N; i++) {
        for (int k = 0; k < K; k++) {
            double top = 0.0, bot = 0.0;
            if (k > 0)
                top = mdot[(size_t)i * (K + 1) + k] * 0.5 * (theta[(size_t)i * K + k - 1] + theta[(size_t)i * K + k]);
            if (k < K - 1)
                bot = mdot[(size_t)i * (K + 1) + k + 1] * 0.5 * (theta[(size_t)i * K + k] + theta[(size_t)i * K + k + 1]);
            tend[(size_t)i * K + k] = -work_c[(size_t)i * K + k] - (bot - top);
        }
    }
}

/* momentum terms that do not involve the pressure gradient:
 * Q_e - G_e K - vertical advection
 *   vadv = [mdot_{e,k+1} (u_{k+1} - u_k) + mdot_{e,k} (u_k - u_{k-1})] / (2 dpi_{e,k})
 * with mdot_e and dpi_e the means of the two cells. */
static void momentum_adv(const or_mesh *h, const or_params *p, const double *u, const double *F,
                         const double *dpi, const double *mdot, double *out,
                         double *ke, double *zeta, double *dpiv, double *qv, double *Q)
{
    const or_mesh_in *m = &h->m;
    const int K = p->K;
    or_kinetic_energy(h, K, u, ke);
    or_curl(h, K, u, zeta);
    or_vertex_mass(h, K, dpi, dpiv);
#pragma omp parallel for schedule(static)
    for (int v = 0; v < m->V; v++)
        for (int k = 0; k < K; k++)
            qv[(size_t)v * K + k] = (zeta[(size_t)v * K + k] + m->fVertex[v]) / dpiv[(size_t)v * K + k];
    or_coriolis(h, K, F, qv, Q);
#pragma omp parallel for schedule(static)
    for (int e = 0; e < m->E; e++) {
        int c1 = m->cells_on_edge[2 * e], c2 = m->cells_on_edge[2 * e + 1];
        for (int k = 0; k < K; k++) {
            size_t x = (size_t)e * K + k;
            double gk = (ke[(size_t)c2 * K + k] - ke[(size_t)c1 * K + k]) / m->dEdge[e];
            double dpie = 0.5 * (dpi[(size_t)c1 * K + k] + dpi[(size_t)c2 * K + k]);
            double va = 0.0;
            if (k < K - 1) {
                double mb = 0.5 * (mdot[(size_t)c1 * (K + 1) + k + 1] + mdot[(size_t)c2 * (K + 1) + k + 1]);
                va += mb * (u[x + 1] - u[x]);
            }
            if (k > 0) {
                double mt = 0.5 * (mdot[(size_t)c1 * (K + 1) + k] + mdot[(size_t)c2 * (K + 1) + k]);
                va += mt * (u[x] - u[x - 1]);
            }
            va /= 2.0 * dpie;
            out[x] = Q[x] - gk - va;
        }
    }
}

/* ------------------------------------------------------------------ */
/* hydrostatic dycore                                                  */
/* ------------------------------------------------------------------ */
/*
 * Column diagnostics (Eq. 8): pi at interfaces pi_t + sigma (pi_s - pi_t),
 * p_k the mean of its two interfaces, theta = Theta/dpi, T = theta (p/p0)^kappa,
 * alpha = R_d T / p, phi_K = 0 at the flat surface and
 * phi_k = phi_{k+1} + alpha_k dpi_k upwards; phi of a layer is the mean of its
 * interfaces.  The PGF is -[alpha_e (p_c2 - p_c1) + (phi_c2 - phi_c1)] / d_e.
 */
static void hydro_pgf(const or_mesh *h, const or_params *p, const double *ps, const double *Theta,
                      double *pgf, double *alpha, double *pmid, double *phim)
{
    const or_mesh_in *m = &h->m;
    const int K = p->K;
    const double kappa = p->rd / p->cp;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < m->N; i++) {
        double phib = p->phis ? p->phis[i] : 0.0;   /* geopotential of the surface (terrain) */
        for (int k = K - 1; k >= 0; k--) {
            size_t x = (size_t)i * K + k;
            double pit = p->ptop + p->sigma[k] * (ps[i] - p->ptop);
            double pib = p->ptop + p->sigma[k + 1] * (ps[i] - p->ptop);
            double dpi = (p->sigma[k + 1] - p->sigma[k]) * (ps[i] - p->ptop);
            double pk = 0.5 * (pit + pib);
            double th = Theta[x] / dpi;
            double T = th * pow(pk / p->p0, kappa);
            double al = p->rd * T / pk;
            double phit = phib + al * dpi;
            pmid[x] = pk;
            alpha[x] = al;
            phim[x] = 0.5 * (phit + phib);
            phib = phit;
        }
    }
#pragma omp parallel for schedule(static)
    for (int e = 0; e < m->E; e++) {
        int c1 = m->cells_on_edge[2 * e], c2 = m->cells_on_edge[2 * e + 1];
        for (int k = 0; k < K; k++) {
            size_t a1 = (size_t)c1 * K + k, a2 = (size_t)c2 * K + k;
            double ae = 0.5 * (alpha[a1] + alpha[a2]);
            pgf[(size_t)e * K + k] = -(ae * (pmid[a2] - pmid[a1]) + (phim[a2] - phim[a1])) / m->dEdge[e];
        }
    }
}

/*
 * One RK3 step of the hydrostatic dry dycore, state (pi_s, Theta = dpi theta, u):
 *   dpi_s/dt = -sum_k D_k (Eq. 3), dTheta/dt from Eq. 4, du/dt from Eq. 5.
 * Stage s: pi_s and Theta are advanced first; the PGF/gravity term then uses
 * them (forward-backward); every other term uses the previous stage's state.
 * With p->no_fb the PGF/gravity term also uses the previous stage's state.
 */
/* Mass fluxes handed to a time-split tracer step (Section 2.3: the tracer's
 * mass flux is accumulated and averaged from the dycore's, Eq. 3): the
 * horizontal flux F [E][K] and the vertical flux mdot [N][K+1] of the last
 * RK stage of every step (the stage that advances the state over the whole
 * dt) are added to Facc and Macc when these are not NULL. */
static void accumulate(size_t n, const double *x, double *acc)
{
    for (size_t j = 0; j < n; j++) acc[j] += x[j];
}

static void hdc_run(const or_mesh *h, const or_params *p, double *ps, double *Theta, double *u, int nsteps,
                    double *Facc, double *Macc)
{
    const or_mesh_in *m = &h->m;
    const int N = m->N, E = m->E, V = m->V, K = p->K;
    const size_t NK = (size_t)N * K, EK = (size_t)E * K, VK = (size_t)V * K;
    double *ps0 = dalloc(N), *Th0 = dalloc(NK), *u0 = dalloc(EK);
    double *dpi = dalloc(NK), *F = dalloc(EK), *D = dalloc(NK), *dps = dalloc(N);
    double *mdot = dalloc((size_t)N * (K + 1)), *theta = dalloc(NK), *dTh = dalloc(NK);
    double *we = dalloc(EK), *wc = dalloc(NK), *adv = dalloc(EK), *ke = dalloc(NK);
    double *zeta = dalloc(VK), *dpiv = dalloc(VK), *qv = dalloc(VK), *Q = dalloc(EK);
    double *pgf = dalloc(EK), *alpha = dalloc(NK), *pmid = dalloc(NK), *phim = dalloc(NK);
    double *psn = dalloc(N), *Thn = dalloc(NK);
    for (int step = 0; step < nsteps; step++) {
        memcpy(ps0, ps, sizeof(double) * N);
        memcpy(Th0, Theta, sizeof(double) * NK);
        memcpy(u0, u, sizeof(double) * EK);
        for (int s = 0; s < 3; s++) {
            double dts = RK3_FRAC[s] * p->dt;
            layer_mass(p, N, ps, dpi);
            mass_flux(m, K, dpi, u, F);
            or_divergence(h, K, F, D);
            column_mass(p, N, D, dps, mdot);
            for (size_t x = 0; x < NK; x++) theta[x] = Theta[x] / dpi[x];
            theta_tendency(h, p, F, theta, mdot, dTh, we, wc);
            momentum_adv(h, p, u, F, dpi, mdot, adv, ke, zeta, dpiv, qv, Q);
            if (s == 2 && Facc) {
                accumulate(EK, F, Facc);
                accumulate((size_t)N * (K + 1), mdot, Macc);
            }
            for (int i = 0; i < N; i++) psn[i] = ps0[i] + dts * dps[i];
            for (size_t x = 0; x < NK; x++) Thn[x] = Th0[x] + dts * dTh[x];
            if (p->no_fb) hydro_pgf(h, p, ps, Theta, pgf, alpha, pmid, phim);
            else hydro_pgf(h, p, psn, Thn, pgf, alpha, pmid, phim);
            for (size_t x = 0; x < EK; x++) u[x] = u0[x] + dts * (adv[x] + pgf[x]);
            memcpy(ps, psn, sizeof(double) * N);
            memcpy(Theta, Thn, sizeof(double) * NK);
        }
    }
    free(ps0); free(Th0); free(u0); free(dpi); free(F); free(D); free(dps); free(mdot); free(theta);
    free(dTh); free(we); free(wc); free(adv); free(ke); free(zeta); free(dpiv); free(qv); free(Q);
    free(pgf); free(alpha); free(pmid); free(phim); free(psn); free(Thn);
}

void or_hdc_run(const or_mesh *h, const or_params *p, double *ps, double *Theta, double *u, int nsteps)
{
    hdc_run(h, p, ps, Theta, u, nsteps, NULL, NULL);
}

void or_hdc_run_flux(const or_mesh *h, const or_params *p, double *ps, double *Theta, double *u, int nsteps,
                     double *Facc, double *Macc)
{
    hdc_run(h, p, ps, Theta, u, nsteps, Facc, Macc);
}

/* Pressure-gradient and gravity term of the hydrostatic model at (pi_s, Theta)
 * (Eq. 5 with Eqs. 8-9; geopotential integrated from the surface value
 * p->phis), exported for tests: pgf [E][K]. */
void or_hdc_pgf(const or_mesh *h, const or_params *p, const double *ps, const double *Theta, double *pgf)
{
    const size_t NK = (size_t)h->m.N * p->K;
    double *alpha = dalloc(NK), *pmid = dalloc(NK), *phim = dalloc(NK);
    hydro_pgf(h, p, ps, Theta, pgf, alpha, pmid, phim);
    free(alpha); free(pmid); free(phim);
}

/* Tendencies of one hydrostatic stage evaluated at (pi_s, Theta, u), exported
 * for tests: dps [N], dTh [N][K], du_adv [E][K] (all momentum terms except the
 * pressure gradient) and mdot [N][K+1]. */
void or_hdc_tendency(const or_mesh *h, const or_params *p, const double *ps, const double *Theta,
                     const double *u, double *dps, double *dTh, double *du_adv, double *mdot)
{
    const or_mesh_in *m = &h->m;
    const int N = m->N, E = m->E, V = m->V, K = p->K;
    const size_t NK = (size_t)N * K, EK = (size_t)E * K, VK = (size_t)V * K;
    double *dpi = dalloc(NK), *F = dalloc(EK), *D = dalloc(NK), *theta = dalloc(NK);
    double *we = dalloc(EK), *wc = dalloc(NK), *ke = dalloc(NK);
    double *zeta = dalloc(VK), *dpiv = dalloc(VK), *qv = dalloc(VK), *Q = dalloc(EK);
    layer_mass(p, N, ps, dpi);
    mass_flux(m, K, dpi, u, F);
    or_divergence(h, K, F, D);
    column_mass(p, N, D, dps, mdot);
    for (size_t x = 0; x < NK; x++) theta[x] = Theta[x] / dpi[x];
    theta_tendency(h, p, F, theta, mdot, dTh, we, wc);
    momentum_adv(h, p, u, F, dpi, mdot, du_adv, ke, zeta, dpiv, qv, Q);
    free(dpi); free(F); free(D); free(theta); free(we); free(wc); free(ke); free(zeta); free(dpiv);
    free(qv); free(Q);
}

/* ------------------------------------------------------------------ */
/* non-hydrostatic dycore (HEVI)                                       */
/* ------------------------------------------------------------------ */

/* equation of state (Eq. 9) with dphi = phi_top - phi_bottom > 0:
 * p = p0 (R_d Theta / (p0 dphi))^gamma, gamma = c_p / c_v */
static double eos(const or_params *p, double Th, double dphi)
{
    double gamma = p->cp / (p->cp - p->rd);
    return p->p0 * pow(p->rd * Th / (p->p0 * dphi), gamma);
}

/* interface mass: half layers either side; the top and bottom interfaces own half a layer */
static double iface_mass(const double *dpi_col, int K, int k)
{
    if (k == 0) return 0.5 * dpi_col[0];
    if (k == K) return 0.5 * dpi_col[K - 1];
    return 0.5 * (dpi_col[k - 1] + dpi_col[k]);
}

/*
 * Advection of an interface field X (w or phi, Eqs. 6-7):
 *   V.grad X = (1/(A_i dpi^_{i,k})) sum_e s l F^_{e,k} (X_nb - X_i)/2
 *   eta_dot dX/deta = [m_{k-1} (X_k - X_{k-1}) + m_k (X_{k+1} - X_k)] / (2 dpi^_k)
 * F^ is the mass flux averaged to the interface (half weights at the top and
 * bottom), m_k the layer mean of the interface mass fluxes; missing layers
 * contribute nothing.
 */
void or_iface_advection(const or_mesh *h, int K, const double *F, const double *dpi, const double *mdot,
                        const double *X, double *out)
{
    const or_mesh_in *m = &h->m;
    const int K1 = K + 1;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < m->N; i++) {
        const double *dcol = dpi + (size_t)i * K;
        const double *md = mdot + (size_t)i * K1;
        for (int k = 0; k <= K; k++) {
            double acc = 0.0;
            for (int j = m->eoc_offset[i]; j < m->eoc_offset[i + 1]; j++) {
                int e = m->edges_on_cell[j];
                double Fh;
                if (k == 0) Fh = 0.5 * F[(size_t)e * K];
                else if (k == K) Fh = 0.5 * F[(size_t)e * K + K - 1];
                else Fh = 0.5 * (F[(size_t)e * K + k - 1] + F[(size_t)e * K + k]);
                acc += h->sgn[j] * m->lEdge[e] * Fh * 0.5 * (X[(size_t)h->coc[j] * K1 + k] - X[(size_t)i * K1 + k]);
            }
            double dh = iface_mass(dcol, K, k);
            double hadv = acc / (m->areaCell[i] * dh);
            double va = 0.0;
            if (k >= 1) va += 0.5 * (md[k - 1] + md[k]) * (X[(size_t)i * K1 + k] - X[(size_t)i * K1 + k - 1]);
            if (k <= K - 1) va += 0.5 * (md[k] + md[k + 1]) * (X[(size_t)i * K1 + k + 1] - X[(size_t)i * K1 + k]);
            out[(size_t)i * K1 + k] = hadv + va / (2.0 * dh);
        }
    }
}

/*
 * Backward-Euler vertical acoustic step of one column (HEVI, Eqs. 6-9).
 * Linearising p in the layer thickness, p+_k = p*_k - C_k (w+_k - w+_{k+1}),
 * C_k = gamma g dt p*_k / dphi*_k; with D_k = g dt / dpi^_k the interior
 * interfaces k = 1..K-1 satisfy
 *   -D_k C_{k-1} w_{k-1} + [1 + D_k (C_{k-1} + C_k)] w_k - D_k C_k w_{k+1}
 *       = w*_k + D_k (p*_k - p*_{k-1}) - g dt,
 * with w_0 = 0 at the rigid lid; then phi = phi* + g dt w above the surface.
 * The surface interface keeps its geopotential (phi_s: the bottom of every
 * layer-thickness difference) and the w given on entry (its kinematic value,
 * surface_w), which the system does not couple to: with phi_K fixed the
 * bottom layer's thickness changes only through w_{K-1}.
 */
static void vertical_solve(const or_params *p, int K, double dts, const double *Th, const double *dpi,
                           double *w, double *phi, double *ws)
{
    const double g = p->grav, gamma = p->cp / (p->cp - p->rd);
    double *ps = ws, *C = ws + K, *sub = ws + 2 * K, *dia = ws + 3 * K, *sup = ws + 4 * K, *rhs = ws + 5 * K,
           *x = ws + 6 * K;
    for (int k = 0; k < K; k++) {
        double dphi = phi[k] - phi[k + 1];
        ps[k] = eos(p, Th[k], dphi);
        C[k] = gamma * g * dts * ps[k] / dphi;
    }
    int n = K - 1;
    for (int r = 0; r < n; r++) {
        int k = r + 1;
        double D = g * dts / iface_mass(dpi, K, k);
        sub[r] = -D * C[k - 1];
        dia[r] = 1.0 + D * (C[k - 1] + C[k]);
        sup[r] = -D * C[k];
        rhs[r] = w[k] + D * (ps[k] - ps[k - 1]) - g * dts;
    }
    if (n > 0) or_thomas(n, sub, dia, sup, rhs, x);
    w[0] = 0.0;
    for (int r = 0; r < n; r++) w[r + 1] = x[r];
    for (int k = 0; k < K; k++) phi[k] = phi[k] + g * dts * w[k];
}

/*
 * Kinematic vertical velocity at the surface (Eq. 7 at the lower boundary,
 * where the vertical mass flux vanishes and phi = phi_s does not change):
 * g w_s = V.grad phi_s, with V.grad phi_s the horizontal part of the interface
 * advection operator at the surface interface (the bottom layer's mass flux
 * at half weight, over half the bottom layer's mass):
 *   w_s,i = sum_e s l_e F_{e,K-1} (phi_s,nb - phi_s,i) / (2 g A_i dpi_{i,K-1}).
 * Zero over a flat surface.  phi [N][K+1] (its bottom interface is phi_s),
 * F [E][K], dpi [N][K]; writes w[i][K].
 */
void or_nh_surface_w(const or_mesh *h, const or_params *p, const double *F, const double *dpi, const double *phi,
                     double *w)
{
    const or_mesh_in *m = &h->m;
    const int K = p->K, K1 = K + 1;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < m->N; i++) {
        double acc = 0.0;
        for (int j = m->eoc_offset[i]; j < m->eoc_offset[i + 1]; j++) {
            int e = m->edges_on_cell[j];
            acc += h->sgn[j] * m->lEdge[e] * F[(size_t)e * K + K - 1] *
                   (phi[(size_t)h->coc[j] * K1 + K] - phi[(size_t)i * K1 + K]);
        }
        w[(size_t)i * K1 + K] = acc / (2.0 * p->grav * m->areaCell[i] * dpi[(size_t)i * K + K - 1]);
    }
}

/* One column of the vertical solve (exported for tests): w, phi [K+1] hold
 * w*, phi* on entry and the implicit solution on return (w_K and phi_K as
 * given). */
void or_nh_column_solve(const or_params *p, double dts, const double *Th, const double *dpi, double *w, double *phi)
{
    double *ws = dalloc((size_t)7 * p->K);
    vertical_solve(p, p->K, dts, Th, dpi, w, phi, ws);
    free(ws);
}

/* NH pressure-gradient force: p from Eq. 9, alpha = dphi/dpi, mu = dp/dpi at
 * interior interfaces (end values copied from the nearest interior one), layer
 * mu and phi as means of the two interfaces:
 *   PGF = -[alpha_e (p_c2 - p_c1) + mu_e (phi_c2 - phi_c1)] / d_e */
static void nh_pgf(const or_mesh *h, const or_params *p, const double *Th, const double *dpi, const double *phi,
                   double *pgf, double *alpha, double *pm, double *mum, double *phim)
{
    const or_mesh_in *m = &h->m;
    const int K = p->K, K1 = K + 1;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < m->N; i++) {
        const double *ph = phi + (size_t)i * K1;
        const double *dp = dpi + (size_t)i * K;
        double pk[512], mu[513];
        for (int k = 0; k < K; k++) {
            double dphi = ph[k] - ph[k + 1];
            pk[k] = eos(p, Th[(size_t)i * K + k], dphi);
            alpha[(size_t)i * K + k] = dphi / dp[k];
            pm[(size_t)i * K + k] = pk[k];
            phim[(size_t)i * K + k] = 0.5 * (ph[k] + ph[k + 1]);
        }
        mu[1] = 1.0;  /* K == 1: a single layer has no interior interface */
        for (int k = 1; k < K; k++) mu[k] = (pk[k] - pk[k - 1]) / iface_mass(dp, K, k);
        mu[0] = mu[1];
        mu[K] = mu[K - 1];
        for (int k = 0; k < K; k++) mum[(size_t)i * K + k] = 0.5 * (mu[k] + mu[k + 1]);
    }
#pragma omp parallel for schedule(static)
    for (int e = 0; e < m->E; e++) {
        int c1 = m->cells_on_edge[2 * e], c2 = m->cells_on_edge[2 * e + 1];
        for (int k = 0; k < K; k++) {
            size_t a1 = (size_t)c1 * K + k, a2 = (size_t)c2 * K + k;
            double ae = 0.5 * (alpha[a1] + alpha[a2]);
            double me = 0.5 * (mum[a1] + mum[a2]);
            pgf[(size_t)e * K + k] = -(ae * (pm[a2] - pm[a1]) + me * (phim[a2] - phim[a1])) / m->dEdge[e];
        }
    }
}

/*
 * One RK3 step of the non-hydrostatic dycore, state (pi_s, Theta, u, w, phi).
 * Stage s: (0) the surface w takes its kinematic value from the stage's
 * mass flux and phi_s (or_nh_surface_w); (1) pi_s and Theta advance with
 * tendencies of the previous stage; (2) w and phi take their explicit
 * advective step w* = w^n + dt_s adv, phi* likewise (the surface keeps phi_s
 * and its w); (3) the implicit column solve turns (w*, phi*) into the stage's
 * w and phi using the new Theta and dpi; (4) u advances with the previous
 * stage's advective terms and the PGF of the new (dpi, Theta, phi).
 */
static void ndc_run(const or_mesh *h, const or_params *p, double *ps, double *Theta, double *u, double *w,
                    double *phi, int nsteps, double *Facc, double *Macc)
{
    const or_mesh_in *m = &h->m;
    const int N = m->N, E = m->E, V = m->V, K = p->K, K1 = K + 1;
    const size_t NK = (size_t)N * K, EK = (size_t)E * K, VK = (size_t)V * K, NK1 = (size_t)N * K1;
    double *ps0 = dalloc(N), *Th0 = dalloc(NK), *u0 = dalloc(EK), *w0 = dalloc(NK1), *phi0 = dalloc(NK1);
    double *dpi = dalloc(NK), *F = dalloc(EK), *D = dalloc(NK), *dps = dalloc(N);
    double *mdot = dalloc(NK1), *theta = dalloc(NK), *dTh = dalloc(NK);
    double *we = dalloc(EK), *wc = dalloc(NK), *adv = dalloc(EK), *ke = dalloc(NK);
    double *zeta = dalloc(VK), *dpiv = dalloc(VK), *qv = dalloc(VK), *Q = dalloc(EK);
    double *pgf = dalloc(EK), *alpha = dalloc(NK), *pm = dalloc(NK), *mum = dalloc(NK), *phim = dalloc(NK);
    double *psn = dalloc(N), *Thn = dalloc(NK), *dpin = dalloc(NK);
    double *aw = dalloc(NK1), *aphi = dalloc(NK1), *wn = dalloc(NK1), *phin = dalloc(NK1);
    for (int step = 0; step < nsteps; step++) {
        memcpy(ps0, ps, sizeof(double) * N);
        memcpy(Th0, Theta, sizeof(double) * NK);
        memcpy(u0, u, sizeof(double) * EK);
        memcpy(w0, w, sizeof(double) * NK1);
        memcpy(phi0, phi, sizeof(double) * NK1);
        for (int s = 0; s < 3; s++) {
            double dts = RK3_FRAC[s] * p->dt;
            layer_mass(p, N, ps, dpi);
            mass_flux(m, K, dpi, u, F);
            or_divergence(h, K, F, D);
            column_mass(p, N, D, dps, mdot);
            for (size_t x = 0; x < NK; x++) theta[x] = Theta[x] / dpi[x];
            theta_tendency(h, p, F, theta, mdot, dTh, we, wc);
            momentum_adv(h, p, u, F, dpi, mdot, adv, ke, zeta, dpiv, qv, Q);
            or_nh_surface_w(h, p, F, dpi, phi, w);
            or_iface_advection(h, K, F, dpi, mdot, w, aw);
            or_iface_advection(h, K, F, dpi, mdot, phi, aphi);
            if (s == 2 && Facc) {
                accumulate(EK, F, Facc);
                accumulate(NK1, mdot, Macc);
            }
            for (int i = 0; i < N; i++) psn[i] = ps0[i] + dts * dps[i];
            for (size_t x = 0; x < NK; x++) Thn[x] = Th0[x] + dts * dTh[x];
            layer_mass(p, N, psn, dpin);
#pragma omp parallel for schedule(static)
            for (int i = 0; i < N; i++) {
                double wsp[7 * 512];
                double *wc_ = wn + (size_t)i * K1, *pc = phin + (size_t)i * K1;
                for (int k = 0; k <= K; k++) {
                    size_t x = (size_t)i * K1 + k;
                    wc_[k] = k == 0 ? 0.0 : k == K ? w[x] : w0[x] - dts * aw[x];
                    pc[k] = (k == K) ? phi0[x] : phi0[x] - dts * aphi[x];
                }
                vertical_solve(p, K, dts, Thn + (size_t)i * K, dpin + (size_t)i * K, wc_, pc, wsp);
            }
            nh_pgf(h, p, Thn, dpin, phin, pgf, alpha, pm, mum, phim);
            for (size_t x = 0; x < EK; x++) u[x] = u0[x] + dts * (adv[x] + pgf[x]);
            memcpy(ps, psn, sizeof(double) * N);
            memcpy(Theta, Thn, sizeof(double) * NK);
            memcpy(w, wn, sizeof(double) * NK1);
            memcpy(phi, phin, sizeof(double) * NK1);
        }
    }
    free(ps0); free(Th0); free(u0); free(w0); free(phi0); free(dpi); free(F); free(D); free(dps); free(mdot);
    free(theta); free(dTh); free(we); free(wc); free(adv); free(ke); free(zeta); free(dpiv); free(qv); free(Q);
    free(pgf); free(alpha); free(pm); free(mum); free(phim); free(psn); free(Thn); free(dpin);
    free(aw); free(aphi); free(wn); free(phin);
}

void or_ndc_run(const or_mesh *h, const or_params *p, double *ps, double *Theta, double *u, double *w,
                double *phi, int nsteps)
{
    ndc_run(h, p, ps, Theta, u, w, phi, nsteps, NULL, NULL);
}

void or_ndc_run_flux(const or_mesh *h, const or_params *p, double *ps, double *Theta, double *u, double *w,
                     double *phi, int nsteps, double *Facc, double *Macc)
{
    ndc_run(h, p, ps, Theta, u, w, phi, nsteps, Facc, Macc);
}

/* ------------------------------------------------------------------ */
/* tracer transport: third-order flux, FCT limiter, RK3                */
/* ------------------------------------------------------------------ */
/*
 * Vertical transport of one column over dt (Eq. 10, the vertical flux
 * divergence), time-split after the horizontal step.  m [K+1] is the mass
 * flux through interface k (between layers k-1 and k), positive towards the
 * surface; m_0 and m_K are taken as zero.  Layer masses:
 *   dpi_new_k = dpih_k - dt (m_{k+1} - m_k).
 * Adaptively implicit split (after Shchepetkin 2015): with the donor layer
 * d(k) (k-1 if m_k >= 0, else k) and the Courant number c = dt |m_k| / dpih_d,
 * the explicit part is mE_k = m_k min(1, 1/(2c)) and the implicit part
 * mI_k = m_k - mE_k.  Both are first-order upwind, the explicit part with the
 * incoming q^h, the implicit part with the new q (backward Euler):
 *   dpi_new_k q_k + dt (GI_{k+1} - GI_k) = dpih_k qh_k - dt (GE_{k+1} - GE_k),
 *   GE_k = mE_k qh_d(k),   GI_k = mI_k q_d(k),
 * a tridiagonal system in q (the same for every tracer) solved with the Thomas
 * algorithm.  q [K][T] holds q^h on entry and the new q on return. */
void or_tracer_vertical_column(int K, int T, double dt, const double *dpih, const double *m, double *q,
                               double *dpi_new)
{
    double *mE = dalloc(K + 1), *mI = dalloc(K + 1);
    double *sub = dalloc(K), *dia = dalloc(K), *sup = dalloc(K), *rhs = dalloc(K), *x = dalloc(K);
    for (int k = 0; k <= K; k++) {
        double mk = (k == 0 || k == K) ? 0.0 : m[k];
        mE[k] = mk;
        if (mk != 0.0) {
            double donor = (mk >= 0.0) ? dpih[k - 1] : dpih[k];
            double c = dt * fabs(mk) / donor;
            if (c > 0.5) mE[k] = mk * (0.5 / c);
        }
        mI[k] = mk - mE[k];
    }
    for (int k = 0; k < K; k++) {
        double mt = (k == 0) ? 0.0 : m[k], mb = (k == K - 1) ? 0.0 : m[k + 1];
        dpi_new[k] = dpih[k] - dt * (mb - mt);
        double at = dt * mI[k], ab = dt * mI[k + 1];
        sub[k] = -fmax(at, 0.0);                                   /* inflow from above */
        dia[k] = dpi_new[k] + fmax(ab, 0.0) + fmax(-at, 0.0);      /* outflow through both interfaces */
        sup[k] = -fmax(-ab, 0.0);                                  /* inflow from below */
    }
    for (int t = 0; t < T; t++) {
        for (int k = 0; k < K; k++) {
            /* explicit upwind fluxes through the top and bottom interfaces */
            double ge_t = 0.0, ge_b = 0.0;
            if (k > 0) ge_t = mE[k] * ((mE[k] >= 0.0) ? q[(size_t)(k - 1) * T + t] : q[(size_t)k * T + t]);
            if (k < K - 1) ge_b = mE[k + 1] * ((mE[k + 1] >= 0.0) ? q[(size_t)k * T + t] : q[(size_t)(k + 1) * T + t]);
            rhs[k] = dpih[k] * q[(size_t)k * T + t] - dt * (ge_b - ge_t);
        }
        or_thomas(K, sub, dia, sup, rhs, x);
        for (int k = 0; k < K; k++) q[(size_t)k * T + t] = x[k];
    }
    free(mE); free(mI); free(sub); free(dia); free(sup); free(rhs); free(x);
}

/*
 * Per stage s with dt_s (Eq. 10, horizontal part; Zalesak 1979 FCT):
 *   dpi_new = dpi^n - dt_s D(F)                              (FP64 continuity)
 *   F^L_e   = F_e q^n_upwind          (upwind cell: c1 if F_e >= 0 else c2)
 *   q^td    = [dpi^n q^n - dt_s D(F^L)] / dpi_new
 *   A_e     = F_e q~_e(q^(s-1)) - F^L_e
 *   q^max/q^min over {q^n, q^td} of the cell and its edge neighbours
 *   P+ = sum max(0, -s l A)/A_i,  P- = sum max(0, s l A)/A_i
 *   Q+ = (q^max - q^td) dpi_new/dt_s,  Q- = (q^td - q^min) dpi_new/dt_s
 *   R+- = min(1, Q/P) if P > 0 else 0
 *   C_e = min(R+_c2, R-_c1) if A_e >= 0 else min(R+_c1, R-_c2)
 *   q^(s) = [dpi^n q^n - dt_s D(F^L + C A)] / dpi_new
 * With fct == 0 the bounds are +-infinity, so R = 1 where P > 0 and the step
 * is the unlimited third-order scheme.
 */
void or_tracer_run(const or_mesh *h, const or_params *p, const double *F, const double *vflux, double *dpi,
                   double *q, int nsteps)
{
    const or_mesh_in *m = &h->m;
    const int N = m->N, E = m->E, K = p->K, T = p->T;
    const size_t NK = (size_t)N * K, EK = (size_t)E * K;
    double *divF = dalloc(NK), *dpin = dalloc(NK);
    double *qn = dalloc(NK), *qs = dalloc(NK), *qtd = dalloc(NK), *FL = dalloc(EK), *Aa = dalloc(EK);
    double *qe = dalloc(EK), *dL = dalloc(NK), *Rp = dalloc(NK), *Rm = dalloc(NK), *Ft = dalloc(EK), *dT = dalloc(NK);
    or_divergence(h, K, F, divF);
    for (int step = 0; step < nsteps; step++) {
        for (int t = 0; t < T; t++) {
            for (size_t x = 0; x < NK; x++) { qn[x] = q[x * T + t]; qs[x] = qn[x]; }
            for (int s = 0; s < 3; s++) {
                double dts = RK3_FRAC[s] * p->dt;
                for (size_t x = 0; x < NK; x++) dpin[x] = dpi[x] - dts * divF[x];
                for (int e = 0; e < E; e++) {
                    int c1 = m->cells_on_edge[2 * e], c2 = m->cells_on_edge[2 * e + 1];
                    for (int k = 0; k < K; k++) {
                        size_t x = (size_t)e * K + k;
                        FL[x] = F[x] * ((F[x] >= 0.0) ? qn[(size_t)c1 * K + k] : qn[(size_t)c2 * K + k]);
                    }
                }
                or_divergence(h, K, FL, dL);
                for (size_t x = 0; x < NK; x++) qtd[x] = (dpi[x] * qn[x] - dts * dL[x]) / dpin[x];
                or_edge_value3(h, K, qs, F, qe);
                for (size_t x = 0; x < EK; x++) Aa[x] = F[x] * qe[x] - FL[x];
#pragma omp parallel for schedule(static)
                for (int i = 0; i < N; i++) {
                    for (int k = 0; k < K; k++) {
                        size_t x = (size_t)i * K + k;
                        double qmax = qn[x] > qtd[x] ? qn[x] : qtd[x];
                        double qmin = qn[x] < qtd[x] ? qn[x] : qtd[x];
                        double Pp = 0.0, Pm = 0.0;
                        for (int j = m->eoc_offset[i]; j < m->eoc_offset[i + 1]; j++) {
                            size_t y = (size_t)h->coc[j] * K + k;
                            if (qn[y] > qmax) qmax = qn[y];
                            if (qtd[y] > qmax) qmax = qtd[y];
                            if (qn[y] < qmin) qmin = qn[y];
                            if (qtd[y] < qmin) qmin = qtd[y];
                            int e = m->edges_on_cell[j];
                            double fo = h->sgn[j] * m->lEdge[e] * Aa[(size_t)e * K + k];
                            if (-fo > 0.0) Pp += -fo;
                            if (fo > 0.0) Pm += fo;
                        }
                        Pp /= m->areaCell[i];
                        Pm /= m->areaCell[i];
                        if (!p->fct) { qmax = INFINITY; qmin = -INFINITY; }
                        double Qp = (qmax - qtd[x]) * dpin[x] / dts;
                        double Qm = (qtd[x] - qmin) * dpin[x] / dts;
                        Rp[x] = (Pp > 0.0) ? fmin(1.0, Qp / Pp) : 0.0;
                        Rm[x] = (Pm > 0.0) ? fmin(1.0, Qm / Pm) : 0.0;
                    }
                }
#pragma omp parallel for schedule(static)
                for (int e = 0; e < E; e++) {
                    int c1 = m->cells_on_edge[2 * e], c2 = m->cells_on_edge[2 * e + 1];
                    for (int k = 0; k < K; k++) {
                        size_t x = (size_t)e * K + k;
                        size_t a1 = (size_t)c1 * K + k, a2 = (size_t)c2 * K + k;
                        double C = (Aa[x] >= 0.0) ? fmin(Rp[a2], Rm[a1]) : fmin(Rp[a1], Rm[a2]);
                        Ft[x] = FL[x] + C * Aa[x];
                    }
                }
                or_divergence(h, K, Ft, dT);
                for (size_t x = 0; x < NK; x++) qs[x] = (dpi[x] * qn[x] - dts * dT[x]) / dpin[x];
            }
            for (size_t x = 0; x < NK; x++) q[x * T + t] = qs[x];
        }
        for (size_t x = 0; x < NK; x++) dpi[x] = dpi[x] - p->dt * divF[x];
        if (vflux) {
            /* vertical step of every column, after the horizontal one */
#pragma omp parallel for schedule(static)
            for (int i = 0; i < N; i++) {
                double dpv[512];
                or_tracer_vertical_column(K, T, p->dt, dpi + (size_t)i * K, vflux + (size_t)i * (K + 1),
                                          q + (size_t)i * K * T, dpv);
                memcpy(dpi + (size_t)i * K, dpv, sizeof(double) * K);
            }
        }
    }
    free(divF); free(dpin); free(qn); free(qs); free(qtd); free(FL); free(Aa); free(qe); free(dL);
    free(Rp); free(Rm); free(Ft); free(dT);
}

/* ------------------------------------------------------------------ */
/* diagnostics                                                          */
/* ------------------------------------------------------------------ */
/* Neumaier-compensated accumulation */
typedef struct { double s, c; } nsum;
static void nadd(nsum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}

/* Area-weighted normalised error norms (Williamson et al. 1992), Eq. 2:
 *   l1 = sum A|x-r| / sum A|r|,  l2 = sqrt(sum A (x-r)^2 / sum A r^2),
 *   linf = max|x-r| / max|r|;  area [n], fields [n][K]. */
void or_norms(int n, int K, const double *area, const double *x, const double *r, double out[3])
{
    nsum a1 = {0, 0}, b1 = {0, 0}, a2 = {0, 0}, b2 = {0, 0};
    double mi = 0.0, mr = 0.0;
    for (int i = 0; i < n; i++)
        for (int k = 0; k < K; k++) {
            size_t j = (size_t)i * K + k;
            double d = x[j] - r[j];
            nadd(&a1, area[i] * fabs(d));
            nadd(&b1, area[i] * fabs(r[j]));
            nadd(&a2, area[i] * d * d);
            nadd(&b2, area[i] * r[j] * r[j]);
            if (fabs(d) > mi) mi = fabs(d);
            if (fabs(r[j]) > mr) mr = fabs(r[j]);
        }
    out[0] = (a1.s + a1.c) / (b1.s + b1.c);
    out[1] = sqrt((a2.s + a2.c) / (b2.s + b2.c));
    out[2] = mi / mr;
}

/*
 * Total energy (J) of a state: kinetic, internal and potential energy of the
 * mass of every layer,
 *   E = (1/g) sum_i A_i sum_k dpi_{i,k} (K_{i,k} + c_v T_{i,k} + phi_{i,k}),
 * with K the cell kinetic energy per unit mass (1/A_i) sum (l d / 4) u^2.
 * Hydrostatic (model 1): dpi from pi_s and sigma, T = theta (p_k/p0)^kappa at
 * the mid-layer pressure, phi_k the mean of the interface geopotentials
 * integrated upwards from phi_s (Eq. 8).  Non-hydrostatic (model 2): p_k from
 * Eq. 9, alpha_k = dphi_k/dpi_k, T = p_k alpha_k / R_d, phi_k the mean of the
 * prognostic interface values, and the vertical kinetic energy adds the
 * mean of w^2/2 at the layer's two interfaces.  Shallow water (model 0):
 *   E = sum_i A_i h_i (K_i + g (h_i/2 + b_i)),
 * the kinetic energy and the potential energy of the column above b.
 * Fields: ps or h [N], Theta [N][K], u [E][K], w and phi [N][K+1], b [N]
 * (NULL where a model has none).  Cells are summed in order (Neumaier).
 */
double or_energy(const or_mesh *h, const or_params *p, int model, const double *ps, const double *Theta,
                 const double *u, const double *w, const double *phi, const double *b)
{
    const or_mesh_in *m = &h->m;
    const int N = m->N, K = model == 0 ? 1 : p->K, K1 = K + 1;
    const double kappa = p->rd / p->cp, cv = p->cp - p->rd;
    double *ke = dalloc((size_t)N * K), *col = dalloc(N);
    or_kinetic_energy(h, K, u, ke);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < N; i++) {
        const double *kc = ke + (size_t)i * K;
        if (model == 0) {
            double bi = b ? b[i] : 0.0;
            col[i] = ps[i] * (kc[0] + p->grav * (0.5 * ps[i] + bi));
            continue;
        }
        double acc = 0.0;
        if (model == 1) {
            double phib = p->phis ? p->phis[i] : 0.0;
            for (int k = K - 1; k >= 0; k--) {
                double dpi = (p->sigma[k + 1] - p->sigma[k]) * (ps[i] - p->ptop);
                double pit = p->ptop + p->sigma[k] * (ps[i] - p->ptop);
                double pib = p->ptop + p->sigma[k + 1] * (ps[i] - p->ptop);
                double pk = 0.5 * (pit + pib);
                double T = Theta[(size_t)i * K + k] / dpi * pow(pk / p->p0, kappa);
                double phit = phib + p->rd * T / pk * dpi;
                acc += dpi * (kc[k] + cv * T + 0.5 * (phit + phib));
                phib = phit;
            }
        } else {
            const double *ph = phi + (size_t)i * K1, *wc = w + (size_t)i * K1;
            for (int k = 0; k < K; k++) {
                double dpi = (p->sigma[k + 1] - p->sigma[k]) * (ps[i] - p->ptop);
                double dphi = ph[k] - ph[k + 1];
                double pk = eos(p, Theta[(size_t)i * K + k], dphi);
                double T = pk * (dphi / dpi) / p->rd;
                double kw = 0.25 * (wc[k] * wc[k] + wc[k + 1] * wc[k + 1]);
                acc += dpi * (kc[k] + kw + cv * T + 0.5 * (ph[k] + ph[k + 1]));
            }
        }
        col[i] = acc / p->grav;
    }
    nsum a = {0, 0};
    for (int i = 0; i < N; i++) nadd(&a, m->areaCell[i] * col[i]);
    free(ke);
    free(col);
    return a.s + a.c;
}

/* sum_i A_i sum_k x_{i,k} (Neumaier) */
double or_area_sum(int n, int K, const double *area, const double *x)
{
    nsum a = {0, 0};
    for (int i = 0; i < n; i++)
        for (int k = 0; k < K; k++) nadd(&a, area[i] * x[(size_t)i * K + k]);
    return a.s + a.c;
}
