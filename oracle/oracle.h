/*
 * FP64 CPU oracle for the mixed-precision icosahedral C-grid dynamical core
 * (Chen et al., "Mixed-Precision Computing in the GRIST Dynamical Core",
 * arXiv 2404.08849).
 *
 * TEST INFRASTRUCTURE ONLY.  This plain, slow, double-precision
 * implementation exists to check the GPU library against.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it;
 * the library never links, calls or includes anything from here, and this
 * file shares no code with it.
 *
 * The paper gives the continuous equations (Section 2.3, Eqs. 3-10) and the
 * scheme names (Section 2.1) but defers the discrete operators to the GRIST
 * description papers.  The discretisation below is the TRiSK C-grid reading
 * (Thuburn et al. 2009; Ringler et al. 2010), Wicker-Skamarock RK3 with a
 * Mesinger forward-backward ordering of each stage, a third-order upwind
 * flux (Skamarock & Gassmann 2011) with a Zalesak (1979) FCT limiter, and a
 * backward-Euler HEVI column solve; each function states its definition.
 *
 * Layouts: cell fields [N][K], edge fields [E][K], vertex fields [V][K],
 * interface fields [N][K+1], tracers [N][K][T]; level index k = 0 at the top.
 */
#ifndef MPDC_ORACLE_H
#define MPDC_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int N, E, V;
    const int *cells_on_edge;     /* [E][2]: c1, c2; n_e points c1 -> c2          */
    const int *vertices_on_edge;  /* [E][2]: v1, v2; t_e = k x n_e points v1 -> v2 */
    const int *eoc_offset;        /* [N+1] CSR offsets                             */
    const int *edges_on_cell;     /* CSR, counter-clockwise                        */
    const int *vertices_on_cell;  /* CSR, vertex j between edges j-1 and j         */
    const int *cells_on_vertex;   /* [V][3] counter-clockwise                      */
    const int *edges_on_vertex;   /* [V][3], edge j joins cells j and j+1          */
    const double *xCell, *xVertex, *xEdge; /* unit vectors [..][3]                 */
    const double *dEdge, *lEdge, *areaCell, *areaVertex, *kiteArea, *fVertex;
    double radius;
} or_mesh_in;

typedef struct {
    int K;                 /* layers                                  */
    int T;                 /* tracers (tracer transport only)         */
    double dt;             /* time step [s]                           */
    double grav, rd, cp, p0, ptop;
    const double *sigma;   /* [K+1] interface sigma, 0 at top, 1 at bottom */
    int fct;               /* 1: FCT limiter on; 0: bounds +-inf (limiter inactive) */
    const double *phis;    /* [N] surface geopotential of the hydrostatic model (NULL: flat) */
    int no_fb;             /* SW and hydrostatic model: 1 = every term of an RK stage from the stage's
                              input state (plain RK3); 0 = forward-backward (mass and Theta first,
                              the pressure-gradient / gravity term from the updated values) */
} or_params;

typedef struct or_mesh or_mesh;

/* Mesh tables (once per mesh). */
or_mesh *or_mesh_build(const or_mesh_in *in);
void or_mesh_free(or_mesh *m);
int or_table_sizes(const or_mesh *m, int *n_trisk);
void or_get_cells_on_cell(const or_mesh *m, int *out);        /* [2E] CSR-aligned */
void or_get_edge_sign(const or_mesh *m, double *out);          /* [2E] s_{e,i}     */
void or_get_vertex_sign(const or_mesh *m, double *out);        /* [3V] s'_{e,v}    */
void or_get_trisk(const or_mesh *m, int *off, int *edge, double *w);
void or_get_hessian(const or_mesh *m, double *w);              /* [2E][6]          */

/* Single operators over K layers (pins and operator-level tests). */
void or_gradient(const or_mesh *m, int K, const double *psi, double *out);
void or_divergence(const or_mesh *m, int K, const double *F, double *out);
void or_curl(const or_mesh *m, int K, const double *u, double *out);
void or_kinetic_energy(const or_mesh *m, int K, const double *u, double *out);
void or_vertex_mass(const or_mesh *m, int K, const double *h, double *out);
void or_perp_flux(const or_mesh *m, int K, const double *F, double *out);
void or_coriolis(const or_mesh *m, int K, const double *F, const double *qv, double *out);
void or_hessian_dir(const or_mesh *m, int K, const double *q, double *out);  /* [2E][K] */
void or_edge_value3(const or_mesh *m, int K, const double *q, const double *F, double *out);
void or_edge_value3_formula(int n, const double *qc1, const double *qc2,
                            const double *h1, const double *h2, const double *d,
                            const double *F, double *out);
/* Advection V.grad X + eta_dot dX/deta of an interface field X [N][K+1]
 * (the w and phi equations, Eqs. 6-7) by the layer mass flux F [E][K] and
 * the interface vertical mass flux mdot [N][K+1], with layer masses dpi
 * [N][K]; out [N][K+1]. */
void or_iface_advection(const or_mesh *m, int K, const double *F, const double *dpi, const double *mdot,
                        const double *X, double *out);
int or_thomas(int n, const double *sub, const double *diag, const double *sup,
              const double *rhs, double *x);

/* Time stepping (in place, FP64 throughout). */
void or_sw_run(const or_mesh *m, const or_params *p, double *h, double *u,
               const double *b, int nsteps);
void or_hdc_run(const or_mesh *m, const or_params *p, double *ps, double *Theta,
                double *u, int nsteps);
void or_ndc_run(const or_mesh *m, const or_params *p, double *ps, double *Theta,
                double *u, double *w, double *phi, int nsteps);
/* vflux [N][K+1]: vertical mass flux through the interfaces (positive towards
 * the surface), or NULL for horizontal transport only. */
void or_tracer_run(const or_mesh *m, const or_params *p, const double *F, const double *vflux,
                   double *dpi, double *q, int nsteps);
void or_tracer_vertical_column(int K, int T, double dt, const double *dpih, const double *m, double *q,
                               double *dpi_new);
/* As or_hdc_run / or_ndc_run, adding the horizontal mass flux [E][K] and the
 * vertical mass flux [N][K+1] of each step's last stage to Facc and Macc. */
void or_hdc_run_flux(const or_mesh *m, const or_params *p, double *ps, double *Theta, double *u, int nsteps,
                     double *Facc, double *Macc);
void or_ndc_run_flux(const or_mesh *m, const or_params *p, double *ps, double *Theta, double *u, double *w,
                     double *phi, int nsteps, double *Facc, double *Macc);

void or_hdc_pgf(const or_mesh *m, const or_params *p, const double *ps, const double *Theta, double *pgf);
void or_hdc_tendency(const or_mesh *m, const or_params *p, const double *ps, const double *Theta,
                     const double *u, double *dps, double *dTh, double *du_adv, double *mdot);
void or_nh_column_solve(const or_params *p, double dts, const double *Th, const double *dpi,
                        double *w, double *phi);
/* Kinematic surface w of the non-hydrostatic model (Eq. 7 at the surface):
 * w[i][K] = V.grad phi_s / g from the layer mass flux F [E][K], layer masses
 * dpi [N][K] and the surface geopotential phi[i][K] (phi [N][K+1]). */
void or_nh_surface_w(const or_mesh *m, const or_params *p, const double *F, const double *dpi, const double *phi,
                     double *w);

/* Diagnostics. */
void or_norms(int n, int K, const double *area, const double *x, const double *ref,
              double out[3]);
double or_area_sum(int n, int K, const double *area, const double *x);
/* Total energy (J) of a state: model 0 shallow water (h, u, b), 1 hydrostatic
 * (pi_s, Theta, u; p->phis), 2 non-hydrostatic (pi_s, Theta, u, w, phi); unused
 * fields may be NULL. */
double or_energy(const or_mesh *m, const or_params *p, int model, const double *ps, const double *Theta,
                 const double *u, const double *w, const double *phi, const double *b);
int or_num_threads(void);
void or_set_num_threads(int n);   /* OpenMP threads of later calls */

#ifdef __cplusplus
}
#endif
#endif
