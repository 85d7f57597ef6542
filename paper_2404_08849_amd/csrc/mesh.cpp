// Mesh validation and operator-table derivation (host, FP64).
//
// The tables are those of the TRiSK discretisation of the hexagonal C-grid
// that the paper's dynamical core uses (Section 2.1): outward edge signs,
// curl signs, the tangential-flux (TRiSK) weights, kinetic-energy and
// divergence weights, and the weights of a quadratic least-squares fit that
// give the second derivative of a cell field along each edge direction (the
// third-order upwind flux of Section 2.1 needs them).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <sstream>

#include "mpdc_internal.h"

namespace mpdc {

namespace {

struct V3 {
    double x, y, z;
};
inline V3 ld(const double *p, long i) { return {p[3 * i], p[3 * i + 1], p[3 * i + 2]}; }
inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 scl(V3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 crs(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline double nrm(V3 a) { return std::sqrt(dot(a, a)); }

std::string msg(const char *what, long i) {
    std::ostringstream o;
    o << what << " (entity " << i << ")";
    return o.str();
}

// Least-squares solve of an m x 5 system (m = 5 or 6) by Householder QR:
// returns the 5 x m pseudo-inverse P (row-major) so that x = P b.
bool qr_pinv(int m, double A[6][5], double P[5][6]) {
    double R[6][5];
    double Qt[6][6];
    std::memcpy(R, A, sizeof(R));
    for (int i = 0; i < 6; i++)
        for (int j = 0; j < 6; j++) Qt[i][j] = (i == j) ? 1.0 : 0.0;
    for (int c = 0; c < 5; c++) {
        double alpha = 0.0;
        for (int r = c; r < m; r++) alpha += R[r][c] * R[r][c];
        alpha = std::sqrt(alpha);
        if (alpha == 0.0) return false;
        if (R[c][c] > 0) alpha = -alpha;
        double v[6] = {0, 0, 0, 0, 0, 0};
        for (int r = c; r < m; r++) v[r] = R[r][c];
        v[c] -= alpha;
        double vv = 0.0;
        for (int r = c; r < m; r++) vv += v[r] * v[r];
        if (vv == 0.0) continue;
        for (int j = 0; j < 5; j++) {
            double s = 0.0;
            for (int r = c; r < m; r++) s += v[r] * R[r][j];
            s = 2.0 * s / vv;
            for (int r = c; r < m; r++) R[r][j] -= s * v[r];
        }
        for (int j = 0; j < m; j++) {
            double s = 0.0;
            for (int r = c; r < m; r++) s += v[r] * Qt[r][j];
            s = 2.0 * s / vv;
            for (int r = c; r < m; r++) Qt[r][j] -= s * v[r];
        }
    }
    // P = R^{-1} (Q^T)_{0..4, :}
    for (int j = 0; j < m; j++) {
        for (int r = 4; r >= 0; r--) {
            double s = Qt[r][j];
            for (int k = r + 1; k < 5; k++) s -= R[r][k] * P[k][j];
            if (R[r][r] == 0.0) return false;
            P[r][j] = s / R[r][r];
        }
    }
    return true;
}

}  // namespace

std::string validate_mesh(const mpdc_mesh_desc *d) {
    const long N = d->nCells, E = d->nEdges, V = d->nVertices;
    if (N < 4 || E < 6 || V < 4) return "mesh too small";
    if (N - E + V != 2) return "Euler characteristic N - E + V is not 2";
    const int32_t *ce = d->cells_on_edge, *ve = d->vertices_on_edge, *off = d->eoc_offset;
    const int32_t *ec = d->edges_on_cell, *vc = d->vertices_on_cell, *cv = d->cells_on_vertex,
                  *ev = d->edges_on_vertex;
    if (!ce || !ve || !off || !ec || !vc || !cv || !ev || !d->xCell || !d->xVertex || !d->xEdge || !d->dEdge ||
        !d->lEdge || !d->areaCell || !d->areaVertex || !d->kiteArea || !d->fVertex)
        return "null array in mesh descriptor";
    if (!(d->radius > 0)) return "radius must be positive";
    for (long e = 0; e < E; e++) {
        for (int s = 0; s < 2; s++) {
            if (ce[2 * e + s] < 0 || ce[2 * e + s] >= N) return msg("cells_on_edge out of range", e);
            if (ve[2 * e + s] < 0 || ve[2 * e + s] >= V) return msg("vertices_on_edge out of range", e);
        }
        if (ce[2 * e] == ce[2 * e + 1]) return msg("edge joins a cell to itself", e);
        if (!(d->dEdge[e] > 0) || !(d->lEdge[e] > 0)) return msg("non-positive edge length", e);
    }
    if (off[0] != 0 || off[N] != 2 * E) return "eoc_offset must start at 0 and end at 2E";
    std::vector<int> seen(E, 0);
    for (long i = 0; i < N; i++) {
        int n = off[i + 1] - off[i];
        if (n < 3 || n > kCellSlots) return msg("cell degree outside 3..6", i);
        if (!(d->areaCell[i] > 0)) return msg("non-positive cell area", i);
        V3 xi = ld(d->xCell, i);
        for (int j = 0; j < n; j++) {
            int e = ec[off[i] + j], v = vc[off[i] + j];
            if (e < 0 || e >= E) return msg("edges_on_cell out of range", i);
            if (v < 0 || v >= V) return msg("vertices_on_cell out of range", i);
            if (ce[2 * e] != i && ce[2 * e + 1] != i) return msg("edges_on_cell lists an edge of another cell", i);
            seen[e]++;
            int ep = ec[off[i] + (j + n - 1) % n];
            bool in_e = (ve[2 * e] == v || ve[2 * e + 1] == v), in_p = (ve[2 * ep] == v || ve[2 * ep + 1] == v);
            if (!in_e || !in_p) return msg("vertex j is not shared by edges j-1 and j", i);
            int vn = vc[off[i] + (j + 1) % n];
            V3 a = sub(ld(d->xVertex, v), xi), b = sub(ld(d->xVertex, vn), xi);
            if (dot(crs(a, b), xi) <= 0) return msg("cell is not counter-clockwise", i);
        }
    }
    for (long e = 0; e < E; e++)
        if (seen[e] != 2) return msg("edge not listed by exactly its two cells", e);
    for (long e = 0; e < E; e++) {
        V3 n = sub(ld(d->xCell, ce[2 * e + 1]), ld(d->xCell, ce[2 * e]));
        V3 t = crs(ld(d->xEdge, e), n);
        V3 dv = sub(ld(d->xVertex, ve[2 * e + 1]), ld(d->xVertex, ve[2 * e]));
        if (dot(t, dv) <= 0) return msg("t_e = k x n_e does not point from v1 to v2", e);
    }
    for (long v = 0; v < V; v++) {
        if (!(d->areaVertex[v] > 0)) return msg("non-positive vertex area", v);
        for (int j = 0; j < 3; j++) {
            int c = cv[3 * v + j], e = ev[3 * v + j];
            if (c < 0 || c >= N) return msg("cells_on_vertex out of range", v);
            if (e < 0 || e >= E) return msg("edges_on_vertex out of range", v);
            if (!(d->kiteArea[3 * v + j] > 0)) return msg("non-positive kite area", v);
            int cn = cv[3 * v + (j + 1) % 3];
            bool joins = (ce[2 * e] == c && ce[2 * e + 1] == cn) || (ce[2 * e] == cn && ce[2 * e + 1] == c);
            if (!joins) return msg("edges_on_vertex[j] does not join cells j and j+1", v);
        }
        V3 a = ld(d->xCell, cv[3 * v]), b = ld(d->xCell, cv[3 * v + 1]), c = ld(d->xCell, cv[3 * v + 2]);
        if (dot(crs(sub(b, a), sub(c, a)), ld(d->xVertex, v)) <= 0) return msg("vertex is not counter-clockwise", v);
    }
    return "";
}

std::string derive_tables(const mpdc_mesh_desc *d, HostTables &t) {
    const long N = d->nCells, E = d->nEdges, V = d->nVertices;
    const int32_t *ce = d->cells_on_edge, *ve = d->vertices_on_edge, *off = d->eoc_offset;
    const int32_t *ec = d->edges_on_cell, *vc = d->vertices_on_cell, *cv = d->cells_on_vertex,
                  *ev = d->edges_on_vertex;
    const int S = kCellSlots;

    // ---- cells: slots, signs, divergence and kinetic-energy weights ----
    t.c_edge.assign(N * S, -1);
    t.c_nbr.assign(N * S, 0);
    t.c_vert.assign(N * S, 0);
    t.c_div.assign(N * S, 0.0);
    t.c_ke.assign(N * S, 0.0);
    t.c_gk.assign(N * S, 0.0);
    t.c_tk.assign(N * S * S, 0.0);
    t.c_area.assign(d->areaCell, d->areaCell + N);
    t.cells_on_cell.assign(2 * E, 0);
    t.edge_sign.assign(2 * E, 0.0);
    std::vector<int> slot_of(2 * E, -1);   // [E][2]: slot of e in c1 / c2
    for (long i = 0; i < N; i++) {
        int n = off[i + 1] - off[i];
        for (int j = 0; j < S; j++) t.c_nbr[i * S + j] = (int)i;
        for (int j = 0; j < n; j++) {
            int e = ec[off[i] + j];
            bool first = (ce[2 * e] == i);
            double s = first ? 1.0 : -1.0;
            int nb = first ? ce[2 * e + 1] : ce[2 * e];
            t.c_edge[i * S + j] = e;
            t.c_nbr[i * S + j] = nb;
            t.c_vert[i * S + j] = vc[off[i] + j];
            t.c_div[i * S + j] = s * d->lEdge[e] / d->areaCell[i];
            t.c_ke[i * S + j] = 0.25 * d->lEdge[e] * d->dEdge[e] / d->areaCell[i];
            t.c_gk[i * S + j] = s / d->dEdge[e];
            t.cells_on_cell[off[i] + j] = nb;
            t.edge_sign[off[i] + j] = s;
            slot_of[2 * e + (first ? 0 : 1)] = j;
        }
        // a pentagon's sixth vertex slot repeats vertex 0, so edge 4 joins slots 4 and 5
        for (int j = n; j < S; j++) t.c_vert[i * S + j] = vc[off[i]];
    }

    // ---- kite fractions R_{i,v}/A_i around each cell, in CSR order ----
    std::vector<double> kfrac(2 * E, 0.0);
    for (long i = 0; i < N; i++) {
        int n = off[i + 1] - off[i];
        for (int j = 0; j < n; j++) {
            int v = vc[off[i] + j];
            int r = (cv[3 * v] == i) ? 0 : (cv[3 * v + 1] == i) ? 1 : (cv[3 * v + 2] == i) ? 2 : -1;
            if (r < 0) return msg("vertices_on_cell and cells_on_vertex disagree", i);
            kfrac[off[i] + j] = d->kiteArea[3 * v + r] / d->areaCell[i];
        }
    }

    // ---- TRiSK: for edge e and each of its cells, the cell's other edges
    //      counter-clockwise from e with w = s_{e,i} s_{e',i} (1/2 - S_j) ----
    t.trisk_off.assign(E + 1, 0);
    t.trisk_edge.clear();
    t.trisk_w.clear();
    t.e_cell.assign(ce, ce + 2 * E);
    t.e_vert.assign(ve, ve + 2 * E);
    t.e_dinv.resize(E);
    t.e_d2.resize(E);
    for (long e = 0; e < E; e++) {
        t.e_dinv[e] = 1.0 / d->dEdge[e];
        t.e_d2[e] = d->dEdge[e] * d->dEdge[e] / 12.0;
        int pos = 0;
        for (int side = 0; side < 2; side++) {
            int i = ce[2 * e + side];
            int n = off[i + 1] - off[i];
            int j0 = slot_of[2 * e + side];
            double s_ei = (side == 0) ? 1.0 : -1.0;
            double acc = 0.0;
            for (int step = 1; step < n; step++) {
                int j = (j0 + step) % n;
                acc += kfrac[off[i] + j];
                int ep = ec[off[i] + j];
                double s_epi = (ce[2 * ep] == i) ? 1.0 : -1.0;
                double w = s_ei * s_epi * (0.5 - acc);
                if (pos >= kTriskSlots) return msg("TRiSK stencil wider than 10 edges", e);
                // cell i's half-stencil row of edge e (slot j0), column slot j,
                // divided by 4 (the two PV means of the kernels' factored sum)
                t.c_tk[(i * S + j0) * S + j] = 0.25 * (w * d->lEdge[ep] / d->dEdge[e]);
                t.trisk_edge.push_back(ep);
                t.trisk_w.push_back(w);
                pos++;
            }
        }
        t.trisk_off[e + 1] = t.trisk_off[e] + pos;
    }

    // ---- quadratic least-squares fit per cell ----
    // Local frame at x_i: local east (or x-axis near the poles) and north;
    // neighbour k sits at arc length r_k along unit bearing b_k.  Fit
    // q_k - q_i = a x + b y + c x^2 + d xy + e y^2 (x, y in units of the mean
    // arc length L); then along a unit direction (u, v)
    // q'' = (2c u^2 + 2d u v + 2e v^2) / L^2 = Hxx u^2 + 2 Hxy u v + Hyy v^2.
    t.c_hess.assign(N * 3 * S, 0.0);
    t.hessian.assign(2 * E * 6, 0.0);
    std::vector<double> bear(2 * E * 2, 0.0);   // per CSR slot: (u, v) bearing of the neighbour
    for (long i = 0; i < N; i++) {
        int n = off[i + 1] - off[i];
        V3 xi = ld(d->xCell, i);
        V3 ref = (std::fabs(xi.z) < 0.9) ? V3{0, 0, 1} : V3{1, 0, 0};
        V3 ex = crs(ref, xi);
        ex = scl(ex, 1.0 / nrm(ex));
        V3 ey = crs(xi, ex);
        double r[6], bu[6], bv[6], L = 0.0;
        for (int k = 0; k < n; k++) {
            V3 xk = ld(d->xCell, t.cells_on_cell[off[i] + k]);
            r[k] = std::atan2(nrm(crs(xi, xk)), dot(xi, xk));
            V3 tg = sub(xk, scl(xi, dot(xk, xi)));
            double tn = nrm(tg);
            bu[k] = dot(tg, ex) / tn;
            bv[k] = dot(tg, ey) / tn;
            bear[2 * (off[i] + k)] = bu[k];
            bear[2 * (off[i] + k) + 1] = bv[k];
            L += r[k];
        }
        L /= n;
        double A[6][5] = {}, P[5][6] = {};
        for (int k = 0; k < n; k++) {
            double x = r[k] / L * bu[k], y = r[k] / L * bv[k];
            A[k][0] = x; A[k][1] = y; A[k][2] = x * x; A[k][3] = x * y; A[k][4] = y * y;
        }
        if (!qr_pinv(n, A, P)) return msg("degenerate quadratic fit", i);
        double Lm = d->radius * L;
        double inv = 1.0 / (Lm * Lm);
        for (int k = 0; k < n; k++) {
            t.c_hess[(i * 3 + 0) * S + k] = 2.0 * P[2][k] * inv;   // Hxx
            t.c_hess[(i * 3 + 1) * S + k] = P[3][k] * inv;         // Hxy
            t.c_hess[(i * 3 + 2) * S + k] = 2.0 * P[4][k] * inv;   // Hyy
        }
        for (int j = 0; j < n; j++) {
            double u = bu[j], v = bv[j];
            for (int k = 0; k < n; k++)
                t.hessian[(off[i] + j) * 6 + k] = t.c_hess[(i * 3 + 0) * S + k] * u * u +
                                                  2.0 * t.c_hess[(i * 3 + 1) * S + k] * u * v +
                                                  t.c_hess[(i * 3 + 2) * S + k] * v * v;
        }
    }
    // per edge: direction of the other cell in each cell's frame, as (u^2, 2uv, v^2)
    t.e_hdir.assign(E * 6, 0.0);
    for (long e = 0; e < E; e++)
        for (int side = 0; side < 2; side++) {
            int i = ce[2 * e + side];
            long sl = off[i] + slot_of[2 * e + side];
            double u = bear[2 * sl], v = bear[2 * sl + 1];
            t.e_hdir[e * 6 + side * 3 + 0] = u * u;
            t.e_hdir[e * 6 + side * 3 + 1] = 2.0 * u * v;
            t.e_hdir[e * 6 + side * 3 + 2] = v * v;
        }

    // per cell slot: the same directions from the cell's side, and -d^2/6
    t.c_hd.assign(N * S * 8, 0.0);
    for (long i = 0; i < N; i++)
        for (int j = 0; j < off[i + 1] - off[i]; j++) {
            const long e = ec[off[i] + j];
            const int side = (ce[2 * e] == i) ? 0 : 1;
            double *h = &t.c_hd[(i * S + j) * 8];
            for (int q = 0; q < 3; q++) {
                h[q] = t.e_hdir[e * 6 + side * 3 + q];
                h[3 + q] = t.e_hdir[e * 6 + (1 - side) * 3 + q];
            }
            h[6] = -2.0 * t.e_d2[e];
        }

    // ---- vertices ----
    t.v_edge.assign(4 * V, 0);
    t.v_cell.assign(4 * V, 0);
    t.v_curl.assign(4 * V, 0.0);
    t.v_kite.assign(4 * V, 0.0);
    t.v_f.assign(d->fVertex, d->fVertex + V);
    t.v_area.assign(d->areaVertex, d->areaVertex + V);
    t.vertex_sign.resize(3 * V);
    for (long v = 0; v < V; v++) {
        for (int j = 0; j < 3; j++) {
            int e = ev[3 * v + j];
            double s = (ve[2 * e + 1] == v) ? 1.0 : -1.0;
            t.vertex_sign[3 * v + j] = s;
            t.v_edge[4 * v + j] = e;
            t.v_cell[4 * v + j] = cv[3 * v + j];
            t.v_curl[4 * v + j] = s * d->dEdge[e] / d->areaVertex[v];
            t.v_kite[4 * v + j] = d->kiteArea[3 * v + j] / d->areaVertex[v];
        }
        t.v_edge[4 * v + 3] = ev[3 * v];   // pad: valid index, zero weight
        t.v_cell[4 * v + 3] = cv[3 * v];
    }
    return "";
}

}  // namespace mpdc
