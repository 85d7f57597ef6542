// Kernel arguments and launchers of the dycore and tracer kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "mpdc_internal.h"

namespace mpdc {

enum { MODEL_SW = MPDC_MODEL_SW, MODEL_HDC = MPDC_MODEL_HDC, MODEL_NDC = MPDC_MODEL_NDC };
enum {
    POLICY_DBL = MPDC_POLICY_DBL,
    POLICY_MIX = MPDC_POLICY_MIX,
    POLICY_MIX_BOX = MPDC_POLICY_MIX_BOX,
    POLICY_MIX_DBL_MASS = MPDC_POLICY_MIX_DBL_MASS,
    POLICY_MIX_F32_DIV = MPDC_POLICY_MIX_F32_DIV,
    POLICY_MIX_PGF32 = MPDC_POLICY_MIX_PGF32,
    POLICY_SGL = MPDC_POLICY_SGL
};
// Variants of the mixed policy inside the FP32 kernel instances (template
// argument VAR): which terms leave the default split.
enum { VAR_MIX = 0, VAR_BOX = 1, VAR_DBL_MASS = 2, VAR_F32_DIV = 3, VAR_PGF32 = 4, VAR_SGL = 5 };
enum { KERNEL_CELL_A = 0, KERNEL_VERTEX = 1, KERNEL_CELL_B = 2, KERNEL_EDGE = 3 };
// largest work-group of the column kernels (keeps 256 VGPRs available per lane)
constexpr int kColumnThreads = 512;

#ifndef MPDC_XCD_REMAP
#define MPDC_XCD_REMAP 1
#endif
// The dispatcher hands work-groups to the eight XCDs in turn (group b to XCD
// b mod 8), and each XCD has its own L2.  Renumbering the groups so that every
// XCD walks one contiguous run of the curve-ordered cells, edges or vertices
// keeps a stencil's neighbours in the L2 of the XCD that reads them.  The map
// is a bijection of [0, gridDim.x): it moves work between XCDs, never changes
// what a lane computes.
constexpr unsigned kXcds = 8;
__device__ __forceinline__ unsigned xcd_block() {
#if MPDC_XCD_REMAP
    const unsigned nb = gridDim.x, b = blockIdx.x;
    const unsigned q = nb / kXcds, r = nb % kXcds, x = b % kXcds;
    return x * q + (x < r ? x : r) + b / kXcds;
#else
    return blockIdx.x;
#endif
}

// Element o of a read-only mesh table through the scalar data cache: where
// the address is the same in every lane (the row of a uniform-cell
// work-group's own cell or edge) the load is a scalar one, into scalar
// registers, with no vector-memory instruction and no LDS.  Tables only
// (never written by a kernel).
template <typename T> __device__ __forceinline__ T sld(const T *p, long o) {
    return ((const __attribute__((address_space(4))) T *)p)[o];
}
template <typename T> __device__ __forceinline__ void sld6(const T *p, long o, T out[6]) {
#pragma unroll
    for (int s = 0; s < 6; s++) out[s] = sld(p, o + s);
}

// Everything one dycore stage reads and writes.  Pointers of another model
// or policy are null.  "_n": state at the start of the step; "_s": state of
// the previous stage; "_o": output state of this stage.
struct StageArgs {
    DevMesh mesh;
    int K, M;
    int cpb;          // cells per work-group of the column kernels
    int flat_block;   // threads per work-group of the flat kernels
    int vpl;          // (k, m) values per lane of this launch (1, 2; flat kernels also 4)
    int store64;      // 1: store the FP64 u and Theta of this stage (0: only their FP32 shadows)
    double dts, grav, rd, cp, p0, ptop, kappa, gamma, inv_p0;
    const double *dsig;  // [K]
    const double *sig;   // [K+1]
    const double *ps_n, *Th_n, *u_n, *w_n, *phi_n;
    const double *ps_s, *Th_s, *u_s, *w_s, *phi_s;
    const float *u32_s, *th32_s;
    double *ps_o, *Th_o, *u_o, *w_o, *phi_o;
    float *u32_o, *th32_o;
    const double *ps_pg; // pi_s (h) of the pressure-gradient term: ps_o (forward-backward) or ps_s
    const double *b;     // SW bottom height [N]
    const double *phis;  // HDC surface geopotential [N] (zero: flat)
    // stage intermediates
    double *dps;         // [N][M]
    double *mdot;        // [N][K+1][M]
    float *mdot32;       // [N][K+1][M] mixed policies: mdot rounded to FP32 for its advective
                         // users (the vertical theta flux of cell_b, the vertical advection of u)
    int mdot64;          // with mdot32: whether cell_a also stores the FP64 mdot (read only by
                         // the tracer mass-flux accumulation)
    void *ke;            // [N][K][M]      (R; FP64 in the boxed variant)
    void *hth;           // [N][3][K][M]   (R)
    void *qv;            // [V][K][M]      (R)
    void *qh;            // [E][2][K][M]   (R) each cell's share of Coriolis - grad K per edge
    double *alpha, *phim, *pm, *mum;   // [N][K][M]
    double *wstar, *phistar;           // [N][K+1][M]
    const int *nh_terrain;   // NDC: nonzero once the surface geopotential varies between cells
                             // (then k_cell_a forms the kinematic surface w; else it is 0)

    template <typename R> __device__ R *ke_out() const { return (R *)ke; }
    template <typename R> __device__ const R *ke_in() const { return (const R *)ke; }
    template <typename R> __device__ R *hth_out() const { return (R *)hth; }
    template <typename R> __device__ const R *hth_in() const { return (const R *)hth; }
    template <typename R> __device__ R *qv_out() const { return (R *)qv; }
    template <typename R> __device__ const R *qv_in() const { return (const R *)qv; }
    template <typename R> __device__ R *qh_out() const { return (R *)qh; }
    template <typename R> __device__ const R *qh_in() const { return (const R *)qh; }
};

// Stencil tables of the cpb columns of a column work-group, staged once in LDS
// (all K*M/L lanes of a column need the same ones).  Byte offsets from the
// start of the area; every region starts on 16 bytes.  rsize is the size of
// the advective precision R; model-specific tables are left out where unused.
struct ColTabLayout {
    size_t ce, cn, cv;    // int [cpb][6]: edges, neighbours, vertices
    size_t ps;            // double [cpb][7][M]: ps_s of the cell (slot 0), then of its neighbours
    size_t psn, dps;      // double [cpb][M]: ps_n and the column mass tendency (cell_b)
    size_t r;             // cell_a: c_div (FP64), c_ke, c_hess; cell_b: c_div, c_gk, c_tk, c_ke
    size_t hd;            // cell_b: c_hd [cpb][6][8]
    size_t bytes;
};
// (32 bytes: a lane's four FP64 values of a row are one aligned 32-byte pack)
__host__ __device__ inline size_t coltab_round(size_t b) { return (b + 31) & ~(size_t)31; }
__host__ __device__ inline ColTabLayout coltab_layout(int model, int which, int cpb, int M, int rsize) {
    ColTabLayout t;
    size_t o = 0;
    t.ce = o; o += coltab_round((size_t)cpb * 24);
    t.cn = o; o += coltab_round((size_t)cpb * 24);
    t.cv = o; o += coltab_round((size_t)cpb * 24);
    t.ps = o; o += coltab_round((size_t)cpb * 7 * M * 8);
    t.psn = o; o += coltab_round((size_t)cpb * M * 8);
    t.dps = o; o += coltab_round((size_t)cpb * M * 8);
    t.r = o;
    // cell_a: c_div in FP64, c_ke and c_hess in R; cell_b: c_div, c_gk, c_tk, c_ke in R
    if (which == KERNEL_CELL_A) o += (size_t)cpb * (6 * 8 + (6 + (model == MODEL_SW ? 0 : 18)) * rsize);
    else o += (size_t)cpb * (6 + 6 + 36 + 6) * rsize;
    o = coltab_round(o);
    t.hd = o;
    if (which == KERNEL_CELL_B && model != MODEL_SW) o += (size_t)cpb * 6 * 8 * rsize;
    t.bytes = coltab_round(o);
    return t;
}

hipError_t launch_stage_kernel(int model, int policy, const StageArgs &a, int which, hipStream_t s);
hipError_t launch_shadows(int model, const StageArgs &a, hipStream_t s);
// hydrostatic column diagnostics (alpha, layer geopotential) of the stage's
// input state (ps_s, Th_s), FP64, for stages without forward-backward ordering
hipError_t launch_column_diag(const StageArgs &a, hipStream_t s);
// relative vorticity at the vertices of an FP64 velocity [E][KM] into out [V][KM] (diagnostics)
hipError_t launch_vorticity(const DevMesh &m, const double *u, double *out, int KM, hipStream_t s);
size_t stage_lds_bytes(int model, int policy, int which, int cpb, int K, int M);
// (k, m) values per lane of the dycore kernels: 2 when K*M splits evenly
int values_per_lane(int K, int M);

// ---- tracer transport ----
enum { TKERNEL_LOW = 0, TKERNEL_LIMIT = 1, TKERNEL_UPDATE = 2 };
// largest work-group of the tracer kernels
constexpr int kTracerThreads = 512;

struct TracerArgs {
    DevMesh mesh;
    int K, T;
    int cpb;           // threads per work-group
    int vpl;           // tracers per lane (1, 2, 4 or 8 (FP32 only), dividing T)
    int fct;
    double dts;
    const double *F;       // [E][K]   prescribed FP64 mass flux
    const double *dpi_n;   // [N][K]   layer mass at the start of the step
    double *dpi_o;         // [N][K]   layer mass after the step (written by the last stage)
    const void *q_n;       // [N][K][T] (R)
    const void *q_s;       // previous stage (R)
    void *q_o;             // this stage (R)
    void *qtd;             // [N][K][T] low-order solution (R)
    void *hq;              // [N][3][K][T] second-derivative coefficients of q_s (R)
    void *rp, *rm;         // [N][K][T] limiter ratios R+ / R- (R)
    const double *vflux;   // [N][K+1] vertical mass flux through the interfaces (vertical step)
    int last_stage;
};

hipError_t launch_tracer_kernel(int policy, const TracerArgs &a, int which, hipStream_t s);
// vertical step of the whole step dt (a.dts), in place on q_o and dpi_o
hipError_t launch_tracer_vertical(int policy, const TracerArgs &a, hipStream_t s);
// columns per work-group of the vertical step (0: a column does not fit the LDS)
int tracer_vert_columns(int K, int T);
// tracer fluxes from a dycore's accumulators over n steps (clears them)
hipError_t launch_couple(double *Facc, double *Macc, double *F, double *vflux, long nF, long nM, long n,
                         hipStream_t s);
// add the last stage's horizontal [E][K] and vertical [N][K+1] mass fluxes
// (a: the arguments of the last stage) to the accumulators (M = 1)
hipError_t launch_flux_acc(int model, int policy, const StageArgs &a, double *Facc, double *Macc, hipStream_t s);

// ---- diagnostics ----
struct DiagArgs {
    const double *area;   // [N]
    const double *x;      // field [n][inner]   FP64 (or null)
    const float *x32;     // field [n][inner]   FP32 (or null)
    const double *ref;    // reference, same layout (or null)
    const double *w;      // optional second factor [n][inner] (tracer mass: dpi), or null
    long n, inner;        // entities and values per entity
    int xs, xo;           // x/ref index = (i*inner + j)*xs + xo (tracer t of T: xs = T, xo = t)
    double offset;        // subtracted from x before the mass sum (pi_t)
    double *partial;      // [nblocks][8]
};
hipError_t launch_diag(const DiagArgs &a, int nblocks, hipStream_t s);
hipError_t launch_nonfinite(const double *x, const float *x32, long n, unsigned long long *partial, int nblocks,
                            hipStream_t s);
hipError_t launch_cfl(const double *u, const double *dinv, long E, long inner, double dt, double *partial,
                      int nblocks, hipStream_t s);

// ---- per-term precision engine of the hydrostatic dycore ----
// bit t of the term mask: term t in FP32 (the MPDC_TERM_* bits of mpdc.h)
enum {
    TERM_MASS_FLUX = MPDC_TERM_MASS_FLUX,
    TERM_DIVERGENCE = MPDC_TERM_DIVERGENCE,
    TERM_KINETIC_ENERGY = MPDC_TERM_KINETIC_ENERGY,
    TERM_VORTICITY = MPDC_TERM_VORTICITY,
    TERM_VERTEX_MASS = MPDC_TERM_VERTEX_MASS,
    TERM_CORIOLIS = MPDC_TERM_CORIOLIS,
    TERM_THETA_FLUX = MPDC_TERM_THETA_FLUX,
    TERM_VERTICAL_ADVECTION = MPDC_TERM_VERTICAL_ADVECTION,
    TERM_COLUMN_DIAG = MPDC_TERM_COLUMN_DIAG,
    TERM_PRESSURE_GRADIENT = MPDC_TERM_PRESSURE_GRADIENT
};
struct TermArgs {
    double *F;       // [E][K] mass flux, then the momentum's advective sum
    double *D;       // [N][K] prefix sums of the divergence, then the theta flux divergence
    double *theta;   // [N][K] theta of the stage's input
    double *pmid;    // [N][K] mid-layer pressure of the updated state
    unsigned mask;   // bit t set: term t in FP32
};
// one RK stage of the hydrostatic model (M = 1) in the per-term precisions
hipError_t launch_term_stage(const StageArgs &a, const TermArgs &x, hipStream_t s);

// ---- total energy of the dycore state (diagnostics) ----
struct EnergyArgs {
    int model, K, M;
    double grav, rd, cp, p0, ptop;
    const double *sig;            // [K+1]
    const double *ps, *Th, *u;    // [N][M] (h for SW), [N][K][M], [E][K][M]
    const double *w, *phi;        // [N][K+1][M] (non-hydrostatic)
    const double *b, *phis;       // [N] SW bottom height, hydrostatic surface geopotential (or null)
    double *out;                  // [N][M] column energy per unit area (J/m^2)
};
hipError_t launch_energy(const DevMesh &m, const EnergyArgs &e, hipStream_t s);

// ---- streaming reference kernels (bandwidth ceiling of the device) ----
// mode 0: read src (one 8-byte word per work-group into dst), 1: write dst,
// 2: copy src to dst; n16 16-byte words, both pointers 16-byte aligned
hipError_t launch_stream(int mode, const void *src, void *dst, long n16, hipStream_t s);
// nh_terrain[0] = 1 if the bottom interface of phi [N][K+1][M] differs between
// cells for any member, else 0 (one work-group; stream-ordered)
hipError_t launch_surface_check(const double *phi, long N, int K, int M, int *flag, hipStream_t s);

}  // namespace mpdc
