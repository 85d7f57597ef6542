/*
 * mpdc -- mixed-precision icosahedral C-grid dynamical core for AMD MI355X.
 *
 * C ABI of the GPU hot path of the mixed-precision GRIST dynamical core
 * (Chen, Zhang, Wang, Liu, Li, Xue: "Mixed-Precision Computing in the GRIST
 * Dynamical Core for Weather and Climate Modelling", arXiv 2404.08849).
 *
 * What the calls compute (paper anchors):
 *  - mpdc_mesh_create: operator tables of the hexagonal/pentagonal
 *    Arakawa-C grid (Section 2.1, Table 1);
 *  - mpdc_dycore_step: the dry dynamical core -- continuity (Eq. 3),
 *    theta_m transport (Eq. 4), momentum (Eq. 5), and for the
 *    non-hydrostatic model the w/phi equations with the equation of state
 *    and an implicit vertical column solve (Eqs. 6-9, HEVI, Section 2.1);
 *    shallow water is the single-layer special case;
 *  - mpdc_tracer_step: flux-form tracer transport (Eq. 10) with a third-order
 *    upwind flux and an FCT limiter (Section 2.1), double-precision mass
 *    continuity (Section 2.3);
 *  - mpdc_diagnostics: global sums and the L1/L2/Linf error norms of
 *    Section 2.2 (Eqs. 1-2).
 * Precision policies (Section 2.3): MPDC_POLICY_DBL computes everything in
 * FP64; MPDC_POLICY_MIX computes the advective terms, the tracer fluxes and
 * the limiter in FP32 and keeps the pressure-gradient force, gravity and
 * geopotential, the vertex mass in the potential vorticity, the implicit
 * vertical solve and the mass sums in FP64.  The prognostic state stays FP64
 * (tracers are FP32 under MIX); initial states are always written in FP64.
 *
 * Conventions
 *  - Every function returning int returns MPDC_OK (0) or a negative error
 *    code; on error no output is modified and mpdc_last_error() (per thread)
 *    describes the failure.  No C++ exception crosses this boundary.
 *  - The library never allocates device memory: the caller passes device
 *    workspaces (pointer + size in bytes, the pointer 256-byte aligned, as
 *    hipMalloc's and torch's allocations are; INVAL otherwise) that must
 *    outlive the handle that uses them.  Host arrays in descriptors are only
 *    read during the call.
 *  - Streams are hipStream_t passed as void*; NULL is the default stream.
 *    Calls are asynchronous on that stream unless stated otherwise.
 *  - Layouts are level-innermost SoA: cell fields [N][K][M], edge fields
 *    [E][K][M], interface fields [N][K+1][M], tracers [N][K][T]; level 0 is
 *    the model top; M is the ensemble member count.
 *  - Indices are int32, zero based.
 */
#ifndef MPDC_H
#define MPDC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define MPDC_OK 0
#define MPDC_E_INVAL (-1)        /* null pointer or bad argument                          */
#define MPDC_E_MESH (-2)         /* invalid mesh (index, Euler number, degree, orientation, area) */
#define MPDC_E_NOMEM (-3)        /* caller workspace too small                            */
#define MPDC_E_DEVICE (-4)       /* HIP runtime error                                     */
#define MPDC_E_NUMERIC (-5)      /* NaN/Inf found by diagnostics                          */
#define MPDC_E_UNSUPPORTED (-6)  /* unsupported combination of options                    */
#define MPDC_E_STATE (-7)        /* call-order error                                      */

/* ---- models and policies ---- */
#define MPDC_MODEL_SW 0          /* single-layer shallow water (h, u)                     */
#define MPDC_MODEL_HDC 1         /* hydrostatic dry dycore (pi_s, Theta, u)               */
#define MPDC_MODEL_NDC 2         /* non-hydrostatic dry dycore (pi_s, Theta, u, w, phi)   */
#define MPDC_MODEL_TRACER 3      /* tracer transport with a prescribed FP64 mass flux     */

#define MPDC_POLICY_DBL 0        /* all FP64                                               */
#define MPDC_POLICY_MIX 1        /* the paper's term split (see above)                     */
/* Variants of MIX (hydrostatic and non-hydrostatic dycore only; otherwise
 * MPDC_E_UNSUPPORTED):
 *  - MIX_BOX: the terms boxed in Eq. 5 as "FP64 compute, FP32 tendency" --
 *    the kinetic energy (from the FP64 velocity) and its gradient, the
 *    vertical advection of u and of theta, and the pressure-gradient
 *    operator L[...] -- are computed in FP64 and rounded to FP32 once, as a
 *    tendency; the rest as MIX;
 *  - MIX_DBL_MASS: the mass flux of the continuity equation (Eq. 3) is formed
 *    in FP64 from the FP64 velocity (the FP32 users take it rounded): the
 *    switch for local mass conservation of Section 2.3 (about 1-2% of the
 *    run time there; its effect is examined in Section 4.4);
 *  - MIX_F32_DIV: the literal reading of Section 2.3 for continuity: the cell
 *    divergence of the FP32 mass flux is accumulated in FP32, so the edge
 *    terms no longer cancel exactly in the global mass sum (compare the
 *    global mass drift of MIX, where the FP32 fluxes are summed in FP64). */
#define MPDC_POLICY_MIX_BOX 2
#define MPDC_POLICY_MIX_DBL_MASS 3
#define MPDC_POLICY_MIX_F32_DIV 4
/* MIX_PGF32 (hydrostatic and non-hydrostatic dycore): the precision-sensitive
 * terms of Section 2.3 -- the column diagnostics of Eqs. 8-9 (pressure,
 * specific volume, geopotential; non-hydrostatic: the equation of state,
 * the implicit column system and its solution, mu) and the pressure-gradient
 * and gravity term of Eq. 5 -- in FP32, as a single-precision model computes
 * them, the rest as MIX.  Over terrain these two large terms nearly cancel
 * (Section 4), which is where FP32 fails. */
#define MPDC_POLICY_MIX_PGF32 5
/* SGL (hydrostatic and non-hydrostatic dycore, tracer transport): every term
 * in FP32 -- the dycores: the reductions of MIX, the FP32 cell divergence of
 * MIX_F32_DIV, the FP32 diagnostics, column solve and pressure-gradient term
 * of MIX_PGF32, and the vertex mass and potential vorticity in FP32; the
 * tracer transport: also the layer-mass continuity, with the mass flux read
 * as FP32 (no vertical tracer step: MPDC_E_UNSUPPORTED for a vertical flux)
 * -- the single-precision configuration the paper starts from (Section 2.2),
 * finds unacceptable (Section 4.1) and times for all three solvers
 * (Table 2).  The dycores' prognostic state is still stored in FP64 and
 * updated with the FP32 tendencies. */
#define MPDC_POLICY_SGL 6
/* TERMS (hydrostatic dycore, one member): the per-term precision table of
 * the iterative precision reduction (Section 2.2, Eqs. 1-2).  Each term of
 * the stage runs in FP32 if its bit is set in mpdc_config.term_fp32, else in
 * FP64: a term in FP32 takes its inputs rounded to FP32 and its result is
 * kept rounded from FP32; the prognostic state stays FP64.  The terms run
 * as separate, unfused kernels (a tool for choosing a split, not the timed
 * path).  No bit set: an all-FP64 stage; the bits of MIX's FP32 terms
 * (MPDC_TERMS_MIX) reproduce the mixed split to FP32 rounding. */
#define MPDC_POLICY_TERMS 7
#define MPDC_TERM_MASS_FLUX 0           /* F = dpi_e u (Eq. 3)                                  */
#define MPDC_TERM_DIVERGENCE 1          /* cell divergence, dpi_s/dt, vertical mass flux (Eq. 3) */
#define MPDC_TERM_KINETIC_ENERGY 2      /* K and -grad K (Eq. 5)                                */
#define MPDC_TERM_VORTICITY 3           /* zeta at the vertices (Eq. 5)                        */
#define MPDC_TERM_VERTEX_MASS 4         /* kite-weighted dpi_v and q = (zeta + f)/dpi_v         */
#define MPDC_TERM_CORIOLIS 5            /* TRiSK PV flux (Eq. 5)                               */
#define MPDC_TERM_THETA_FLUX 6          /* third-order theta_m flux and its divergence (Eq. 4) */
#define MPDC_TERM_VERTICAL_ADVECTION 7  /* vertical advection of u and theta (Eqs. 4-5)        */
#define MPDC_TERM_COLUMN_DIAG 8         /* pressure, specific volume, geopotential (Eqs. 8-9)  */
#define MPDC_TERM_PRESSURE_GRADIENT 9   /* pressure-gradient force and gravity (Eq. 5)         */
#define MPDC_TERM_COUNT 10
#define MPDC_TERMS_MIX ((1u << MPDC_TERM_MASS_FLUX) | (1u << MPDC_TERM_KINETIC_ENERGY) | \
                        (1u << MPDC_TERM_VORTICITY) | (1u << MPDC_TERM_CORIOLIS) |           \
                        (1u << MPDC_TERM_THETA_FLUX) | (1u << MPDC_TERM_VERTICAL_ADVECTION))

/* ---- state fields for mpdc_state_write / mpdc_state_read (FP64 in and out) ---- */
#define MPDC_FIELD_H 0           /* SW fluid depth h          [N][M]        */
#define MPDC_FIELD_PS 1          /* surface pressure pi_s     [N][M]        */
#define MPDC_FIELD_THETA 2       /* Theta = dpi theta_m       [N][K][M]     */
#define MPDC_FIELD_U 3           /* normal velocity u         [E][K][M]     */
#define MPDC_FIELD_W 4           /* vertical velocity w       [N][K+1][M]: 0 at the lid (k = 0); at
                                    the surface (k = K) each stage sets the kinematic value
                                    V.grad phi_s / g of its flow (Eq. 7 at the surface, where the
                                    vertical mass flux vanishes), zero over a flat surface */
#define MPDC_FIELD_PHI 5         /* geopotential phi          [N][K+1][M]: its surface entry (k = K)
                                    is the surface geopotential phi_s (NDC terrain), which the steps
                                    keep fixed */
#define MPDC_FIELD_B 6           /* SW bottom height b        [N]           */
#define MPDC_FIELD_TR_FLUX 7     /* tracer mass flux F        [E][K]        */
#define MPDC_FIELD_TR_DPI 8      /* tracer layer mass dpi     [N][K]        */
#define MPDC_FIELD_TR_Q 9        /* tracer mixing ratios q    [N][K][T]     */
#define MPDC_FIELD_TR_VFLUX 10   /* tracer vertical mass flux [N][K+1]: through interface k (between
                                    layers k-1 and k), positive towards the surface; the lid and surface
                                    entries are ignored.  Writing it (or mpdc_tracer_couple) turns on the
                                    vertical step of mpdc_tracer_step */
#define MPDC_FIELD_VORT 12       /* read-only (state_read, diagnostics): relative vorticity at the
                                    vertices [V][K][M], (1/A_v) sum s' d u of the FP64 velocity; with
                                    the surface pressure it makes the error measure E of Eqs. 1-2 */
#define MPDC_FIELD_PHIS 11       /* HDC surface geopotential phi_s [N] (terrain; zero = flat surface,
                                    the default), shared by the members; the hydrostatic geopotential
                                    is integrated upwards from it (Eq. 8) */

/* ---- mesh tables exported for checks (mpdc_mesh_get_table) ---- */
#define MPDC_TABLE_CELLS_ON_CELL 0   /* int32 [2E], aligned with edges_on_cell            */
#define MPDC_TABLE_EDGE_SIGN 1       /* double [2E], s_{e,i} = +1 if i = c1(e) else -1    */
#define MPDC_TABLE_VERTEX_SIGN 2     /* double [V][3], s'_{e,v} = +1 if v = v2(e) else -1 */
#define MPDC_TABLE_TRISK_OFFSET 3    /* int32 [E+1]                                        */
#define MPDC_TABLE_TRISK_EDGE 4      /* int32 [n], n = TRISK_OFFSET[E]                     */
#define MPDC_TABLE_TRISK_WEIGHT 5    /* double [n], w_{e,e'}                              */
#define MPDC_TABLE_HESSIAN 6         /* double [2E][6], directional 2nd-derivative weights */

typedef struct {
    int32_t nCells, nEdges, nVertices;
    const int32_t *cells_on_edge;     /* [E][2]  c1, c2; the normal n_e points c1 -> c2          */
    const int32_t *vertices_on_edge;  /* [E][2]  v1, v2; t_e = k x n_e points v1 -> v2           */
    const int32_t *eoc_offset;        /* [N+1]   CSR offsets into the two lists below             */
    const int32_t *edges_on_cell;     /* [2E]    counter-clockwise                                */
    const int32_t *vertices_on_cell;  /* [2E]    vertex j lies between edges j-1 and j            */
    const int32_t *cells_on_vertex;   /* [V][3]  counter-clockwise                                */
    const int32_t *edges_on_vertex;   /* [V][3]  edge j joins cells j and j+1                     */
    const double *xCell, *xVertex, *xEdge;  /* unit position vectors [..][3]                     */
    const double *dEdge;              /* [E] cell-to-cell arc length (m)                          */
    const double *lEdge;              /* [E] vertex-to-vertex arc length (m)                      */
    const double *areaCell;           /* [N] (m^2)                                                */
    const double *areaVertex;         /* [V] (m^2)                                                */
    const double *kiteArea;           /* [V][3] area shared by vertex v and cell cells_on_vertex[v][j] */
    const double *fVertex;            /* [V] Coriolis parameter (1/s)                             */
    double radius;                    /* sphere radius (m)                                        */
} mpdc_mesh_desc;

typedef struct {
    int32_t model;        /* MPDC_MODEL_*                                                   */
    int32_t policy;       /* MPDC_POLICY_*                                                  */
    int32_t K;            /* layers (1 for SW; >= 2 for NDC)                                */
    int32_t M;            /* ensemble members batched member-innermost (>= 1)               */
    int32_t T;            /* tracers (TRACER model)                                         */
    int32_t fct;          /* tracer limiter: 1 on (default), 0 off (bounds +-inf)           */
    double dt;            /* time step (s)                                                  */
    double grav, rd, cp, p0, ptop;  /* g, R_d, c_p, reference and model-top pressure       */
    const double *sigma;  /* [K+1] sigma at interfaces, 0 at the top, 1 at the surface      */
    int32_t accumulate_flux; /* HDC/NDC with M = 1: 1 = sum each step's last-stage horizontal and
                                vertical mass fluxes for mpdc_tracer_couple (0 otherwise)         */
    int32_t forward_backward_off; /* 0 (default): forward-backward stages -- the pressure-gradient
                                (gravity) term of each RK stage uses the mass and Theta that stage
                                has just advanced (Section 2.1: the hydrostatic solver's Mesinger
                                forward-backward scheme); 1: every term of a stage uses the
                                stage's input state (plain RK3).  SW and HDC with the policies
                                DBL, MIX, MIX_BOX, MIX_DBL_MASS, MIX_F32_DIV only (the
                                non-hydrostatic solver's HEVI ordering has no such switch);
                                otherwise MPDC_E_UNSUPPORTED                                     */
    int32_t term_fp32;    /* MPDC_POLICY_TERMS: bit MPDC_TERM_* set = that term in FP32; must be
                             zero for every other policy                                    */
    int32_t reserved[5];  /* must be zero                                                   */
} mpdc_config;

#define MPDC_DIAG_MAX_TRACERS 16  /* per-tracer entries of mpdc_diag */

typedef struct {
    double mass;          /* sum_i A_i h_i (SW) or sum_i A_i (pi_s - pi_t) summed over members */
    double mass_tracer[MPDC_DIAG_MAX_TRACERS];  /* sum A dpi q per tracer                 */
    double min, max;      /* of ref_field, the field named in mpdc_diagnostics              */
    double l1, l2, linf;  /* area-weighted normalised errors vs the reference (if given)    */
    int64_t nonfinite;    /* NaN/Inf count over every prognostic field                      */
    double cfl_max;       /* dycore: largest |u_e| dt / d_e (NaN if u holds one); tracer: 0    */
    double energy;        /* dycore: total energy (J) summed over members -- kinetic, internal
                             and potential energy of every layer's mass,
                             (1/g) sum_i A_i sum_k dpi (K + c_v T + phi), with K the cell
                             kinetic energy (1/A) sum (l d/4) u^2, phi the layer mean of the
                             interface geopotentials (hydrostatic: integrated from phi_s;
                             non-hydrostatic: prognostic, plus the layer mean of w^2/2);
                             shallow water: sum_i A_i h (K + g (h/2 + b)); tracer: 0     */
    double tracer_min[MPDC_DIAG_MAX_TRACERS], tracer_max[MPDC_DIAG_MAX_TRACERS];
                          /* per tracer over every cell and level (tracer model)         */
} mpdc_diag;

typedef struct mpdc_mesh mpdc_mesh;
typedef struct mpdc_state mpdc_state;

/* Bytes of device workspace mpdc_mesh_create needs for this mesh (0 if the
 * descriptor is unusable). */
size_t mpdc_mesh_workspace_bytes(const mpdc_mesh_desc *d);

/* Host-only check of a mesh description: the validation and table
 * derivation of mpdc_mesh_create with no device access.  Returns MPDC_OK or
 * MPDC_E_MESH / MPDC_E_INVAL with the reason in mpdc_last_error(). */
int mpdc_mesh_check(const mpdc_mesh_desc *d);

/* Validate the mesh (index ranges, N - E + V = 2, cell degree 5/6, degree-3
 * vertices, counter-clockwise orientation, positive lengths and areas),
 * derive its operator tables in FP64 on the host (signs, cells-on-cell, TRiSK
 * lists and weights, quadratic-fit second-derivative weights) with FP32
 * copies, and upload them into dev_ws (ws_bytes >= mpdc_mesh_workspace_bytes)
 * on stream s.  *out receives a handle; the descriptor may be freed after the
 * call returns.  Errors: INVAL, MESH, NOMEM, DEVICE. */
int mpdc_mesh_create(const mpdc_mesh_desc *d, void *dev_ws, size_t ws_bytes, void *stream,
                     mpdc_mesh **out);

/* Copy one derived table (MPDC_TABLE_*) to host memory; synchronous.
 * bytes must equal the table size (errors: INVAL). */
int mpdc_mesh_get_table(const mpdc_mesh *m, int table_id, void *host_dst, size_t bytes);
size_t mpdc_mesh_table_bytes(const mpdc_mesh *m, int table_id);
void mpdc_mesh_destroy(mpdc_mesh *m);

/* Device workspace needed by a state of this configuration (0 if unsupported). */
size_t mpdc_state_workspace_bytes(const mpdc_mesh *m, const mpdc_config *c);

/* Create a state (fields zero-initialised asynchronously on the mesh's stream).
 * The mesh must outlive the state.  Errors: INVAL, UNSUPPORTED, NOMEM, DEVICE. */
int mpdc_state_create(const mpdc_mesh *m, const mpdc_config *c, void *dev_ws, size_t ws_bytes,
                      mpdc_state **out);

/* Write a field (MPDC_FIELD_*) from FP64 data on the host (src_on_device = 0)
 * or device; the library converts to its storage precision and regenerates
 * the FP32 shadows.  bytes must equal the field's FP64 size.  Errors: INVAL
 * (field not part of the model, wrong size, or MPDC_FIELD_VORT, which is
 * derived), UNSUPPORTED (MPDC_FIELD_TR_VFLUX with K x T too large for the
 * vertical step), DEVICE.  Synchronous for host sources. */
int mpdc_state_write(mpdc_state *st, int field_id, const void *src, int src_on_device, size_t bytes,
                     void *stream);

/* Read a field back as FP64 into host (dst_on_device = 0; synchronous) or
 * device memory (asynchronous).  MPDC_FIELD_VORT is computed from the current
 * velocity on the fly (it uses the state's stage scratch, so it must not run
 * concurrently with a step of the same state). */
int mpdc_state_read(mpdc_state *st, int field_id, void *dst, int dst_on_device, size_t bytes,
                    void *stream);

/* Advance the dycore (SW, HDC or NDC) by nsteps RK3 steps of dt.  Each stage
 * updates the mass and Theta first and uses them in the pressure-gradient
 * term (forward-backward; see mpdc_config.forward_backward_off).
 * Asynchronous.  Errors: INVAL, STATE, DEVICE. */
int mpdc_dycore_step(mpdc_state *st, int nsteps, void *stream);

/* Advance the tracers (TRACER model) by nsteps RK3 steps with the FCT limiter
 * applied in every stage (horizontal part of Eq. 10).  Once a vertical mass
 * flux is set, each step ends with the vertical part of Eq. 10 over the whole
 * dt, time-split (Section 2.1: adaptively implicit in the vertical): the
 * layer mass loses dt times the flux divergence; each interface flux splits
 * into an explicit part capped at a Courant number of 1/2 (of its upwind
 * layer) and an implicit remainder, both first-order upwind, the implicit one
 * solved per column (tridiagonal, FP64).  Asynchronous.  Errors: INVAL,
 * STATE, DEVICE. */
int mpdc_tracer_step(mpdc_state *st, int nsteps, void *stream);

/* Time-split coupling of the tracer transport to the dycore (Section 2.1;
 * Section 2.3: the tracer's mass flux is accumulated and averaged from the
 * dycore's and used in FP64).  The dycore state (HDC or NDC, created with
 * accumulate_flux = 1) sums, over its steps, the horizontal mass flux of each
 * step's last RK stage exactly as that stage's divergence used it (FP32 values
 * under the mixed policies, FP64 under DBL and MIX_DBL_MASS) and that stage's
 * vertical mass flux.  This call sets the tracer state's horizontal flux
 * (MPDC_FIELD_TR_FLUX) and vertical flux (MPDC_FIELD_TR_VFLUX) to those sums
 * divided by the number of steps n, in FP64, and clears the sums.  A tracer
 * step of n times the dycore's dt then moves each layer mass exactly as the n
 * dycore steps did (up to rounding).  Requirements: same mesh handle and K,
 * tracer dt = n x dycore dt.  Asynchronous on stream.  Errors: INVAL (wrong
 * models, mesh, K or dt), STATE (no accumulation or no step since the last
 * coupling), UNSUPPORTED (K x T too large for the vertical step), DEVICE. */
int mpdc_tracer_couple(mpdc_state *tracer, mpdc_state *dycore, void *stream);

/* Deterministic FP64 reductions over the state: global mass, total energy,
 * tracer masses and per-tracer min/max, NaN/Inf count, min/max of the field
 * ref_field, and (if ref_dev is not NULL) the normalised L1/L2/Linf errors of
 * ref_field against the FP64 device array ref_dev of the same layout
 * (Section 2.2, Eq. 2; cell fields weighted by the cell areas,
 * MPDC_FIELD_VORT by the dual-cell areas, edge fields unweighted).  ref_dev
 * is borrowed for the call.  Synchronous.  Returns MPDC_E_NUMERIC (with *out
 * filled) if a NaN/Inf is present, and MPDC_E_UNSUPPORTED (nothing written)
 * for a tracer state with more than MPDC_DIAG_MAX_TRACERS tracers.  The
 * energy uses the state's stage scratch, so it must not run concurrently
 * with a step of the same state. */
int mpdc_diagnostics(mpdc_state *st, const void *ref_dev, int ref_field, mpdc_diag *out, void *stream);

/* Capture one dycore or tracer step into a HIP graph and replay it for later
 * steps (enable != 0), or go back to direct launches (enable == 0).  Results
 * are bitwise identical either way.  The stream passed to the step calls must
 * not be the legacy default stream while graphs are enabled. */
int mpdc_set_graph(mpdc_state *st, int enable);

/* Launch shape of all the state's kernels: cells per work-group for the
 * column kernels (0 = default) and threads per work-group for the flat
 * kernels (0 = 256).  Any legal shape gives bitwise identical results.
 * Errors: INVAL (a work-group over 512 column lanes or 64 KiB of LDS, or a
 * thread count that is not a multiple of 64 up to 1024, 512 for tracers). */
int mpdc_set_launch(mpdc_state *st, int cells_per_block, int flat_block);

/* Launch shape of one kernel class (ids as for mpdc_time_kernel):
 * values_per_lane = (level, member) values a lane computes -- 1 or 2 for the
 * column kernels (also 4 for an ensemble in the FP32 policies, with one cell
 * per work-group; the default for hydrostatic and shallow-water ensembles of
 * a multiple of four members in those policies), 1, 2 or 4 for the flat
 * kernels, 1, 2, 4 or (mixed policy) 8 tracers for the
 * tracer kernels; it must divide K (M == 1), M (M > 1) or T; 0 = default --
 * and group = cells per work-group (column kernels) or threads per
 * work-group (others; for the tracer kernels also 1: one cell per
 * work-group, K T / values_per_lane <= 512 threads), 0 = keep.  Results are
 * bitwise identical for every legal shape.  Errors: INVAL. */
int mpdc_set_kernel_launch(mpdc_state *st, int kernel_id, int values_per_lane, int group);
int mpdc_get_kernel_launch(const mpdc_state *st, int kernel_id, int *values_per_lane, int *group);

/* Time nreps launches of one kernel class (0 = first cell kernel, 1 = vertex,
 * 2 = second cell kernel, 3 = edge/momentum kernel; tracer: 0..2 its three
 * passes) of stage 1 on stream with HIP events; *ms_avg receives the mean
 * duration.  The state is advanced by nothing (inputs are not modified).  */
int mpdc_time_kernel(mpdc_state *st, int kernel_id, int nreps, void *stream, double *ms_avg);

/* Run nsteps steps with direct launches and a HIP event between consecutive
 * launches on stream, and return per kernel class (ids as above) the summed
 * duration in ms (ms_total[4]) and the launch count (launches[4]); the
 * tracer uses the first three entries for its horizontal kernels and the
 * fourth for the vertical step (zero without a vertical flux).  The state
 * advances by nsteps exactly as with mpdc_dycore_step / mpdc_tracer_step. */
int mpdc_profile_steps(mpdc_state *st, int nsteps, void *stream, double *ms_total, int *launches);

/* Autotuner (the tuned launch shapes of the batched workloads): for each
 * kernel class in launch order, time every legal (values per lane,
 * work-group) pair with mpdc_time_kernel (so the state is not advanced) and
 * keep the fastest; mpdc_get_kernel_launch reads the choice back.  Results
 * stay bitwise identical whatever is chosen.  cache_path (may be NULL: no
 * cache) names a text file of stored choices, one line per configuration
 * keyed by the device (architecture, compute units), the library version,
 * the model, policy, mesh counts, K, M, T and the stage ordering: if it holds
 * a legal choice for this configuration, that choice is applied without
 * timing anything; otherwise the tuned choice replaces or adds that line (the
 * file is rewritten through a temporary file and a rename; concurrent
 * writers of one file may lose each other's lines).  Synchronous.  Errors:
 * INVAL (null state; the cache cannot be written -- the tuned shapes are
 * applied all the same), DEVICE. */
int mpdc_autotune(mpdc_state *st, const char *cache_path, void *stream);

/* Algorithmic HBM bytes of one launch of a kernel class (same ids; mean over
 * the three RK stages; tracer id 3: the vertical step, once per step) and of
 * one whole step, from the arrays each kernel must read and write once. */
double mpdc_kernel_bytes(const mpdc_state *st, int kernel_id);
double mpdc_step_bytes(const mpdc_state *st);

/* Algorithmic HBM bytes of one launch of a kernel class in RK stage `stage`
 * (0, 1 or 2; the tracer's vertical step: its once-per-step figure for any
 * stage).  Stages differ where one reads or writes arrays the others do not:
 * the first reads the step-start state once for both roles, and the mixed
 * policies that read only FP32 shadows (MIX, MIX_F32_DIV, MIX_PGF32, SGL)
 * store the FP64 u and Theta in the last stage only.  mpdc_time_kernel times
 * the first stage's launch (stage = 0 here).  Returns 0 for a bad id or stage. */
double mpdc_stage_kernel_bytes(const mpdc_state *st, int kernel_id, int stage);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the error
 * norms of mpdc_diagnostics without a state or a workspace.  Over the FP64
 * device arrays x and ref [n][inner] and the optional weights [n] (NULL:
 * unweighted), out[0..4] receives the normalised L1, L2 and Linf of x
 * against ref (sum w|x - r| / sum w|r|, sqrt(sum w (x - r)^2 / sum w r^2),
 * max|x - r| / max|r|) and the min and max of x.  The per-work-group partial
 * sums live in a static device array of 1024 x 9 doubles (72 KiB), which
 * each GPU the library runs on holds until the process ends; the reduction
 * strides over any n x inner with at most 1024 work-groups, so every size
 * fits it.  Nothing is allocated on the device.  Every call on one GPU shares
 * that array: calls that overlap on one GPU (several streams or threads)
 * race.  Synchronous on stream.  Errors: INVAL (null pointer, n or inner
 * zero, n x inner overflowing), DEVICE. */
int mpdc_error_norms_noalloc(const double *x, const double *ref, const double *weight, size_t n, size_t inner,
                             double *out, void *stream);

/* Measurement utility, not a step of the method: the device's streaming
 * bandwidth, which the stencil kernels' achieved bandwidth is read against.
 * Times nreps launches of a plain streaming kernel over `bytes` bytes (a
 * positive multiple of 16; dst and src 16-byte aligned device buffers of at
 * least that size) on stream with HIP events, after one untimed launch;
 * *ms_avg receives the mean duration.  mode 0 reads src (and stores one
 * 8-byte word per 16 KiB read at the start of dst), 1 writes dst (src may be
 * NULL), 2 copies src to dst; each lane moves four 16-byte words.
 * Synchronous.  Errors: INVAL, DEVICE. */
int mpdc_stream_time(int mode, void *dst, const void *src, size_t bytes, int nreps, void *stream,
                     double *ms_avg);

void mpdc_state_destroy(mpdc_state *st);

const char *mpdc_strerror(int code);
const char *mpdc_last_error(void);
const char *mpdc_version(void);

#ifdef __cplusplus
}
#endif
#endif
