// HIP kernels of the dry dynamical core for gfx950 (MI355X).
//
// One RK3 stage of the shallow-water (SW), hydrostatic (HDC) and
// non-hydrostatic (NDC) C-grid dycore, written for a level- and
// member-innermost layout ([entity][k][m]).  Each lane owns L consecutive
// (k, m) values of one entity (L = 2 whenever K*M allows it), so every
// stencil gather is an L-wide vector load of a contiguous run and the
// per-entity table lookups are shared by L values.  With M == 1 the L values
// are consecutive levels; with M > 1 they are consecutive members of one
// level.
//
// Per stage (tendencies from the previous stage y^(s-1), base state y^n):
//   cell_a  (cell columns)  divergence of the mass flux, column mass tendency
//                           and vertical mass flux (Eq. 3, LDS prefix sum),
//                           kinetic energy, second derivatives of theta;
//                           NDC: explicit advective step of w and phi (Eqs. 6-7);
//                           SW: the depth update
//   vertex  (vertex x km)   vorticity, FP64 vertex mass, potential vorticity
//   cell_b  (cell columns)  each cell's share of the Coriolis and KE-gradient
//                           terms of its six edges (TRiSK, Eq. 5), theta_m
//                           flux-form transport (Eq. 4, third-order upwind) and
//                           the mass/Theta update; then the FP64 column
//                           diagnostics of the updated state: pressure, alpha
//                           and the hydrostatic geopotential (Eq. 8, LDS scan),
//                           or for NDC the equation of state (Eq. 9) and the
//                           implicit vertical acoustic solve (HEVI)
//   edge    (edge x km)     adds the two cells' shares, vertical advection of
//                           u, FP64 pressure-gradient and gravity term (Eq. 5),
//                           RK update of u
// The TRiSK sum of an edge runs over the other edges of its two cells, so it
// splits exactly into one partial sum per cell; a cell forms both partial
// sums of all its edges from its own six fluxes and six vertex PVs, which
// replaces a ten-edge indirect gather per edge-level.  The mass flux
// F = dpi_e u is recomputed from u and the 2-D surface pressure wherever it is
// needed instead of being stored.
//
// Template parameter R is the arithmetic type of the advective terms:
// double for the all-FP64 policy, float for the mixed policy.  Everything
// the mixed policy keeps in FP64 (mass sums, vertex mass and the PV
// division, pressure gradient, gravity/geopotential, the column solve, the
// state update) is double in both instantiations.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "dycore_kernels.h"

namespace mpdc {

template <typename R> __device__ __forceinline__ const R *pick(const double *d, const float *f);
template <> __device__ __forceinline__ const double *pick<double>(const double *d, const float *) { return d; }
template <> __device__ __forceinline__ const float *pick<float>(const double *, const float *f) { return f; }

template <typename T, int L> struct alignas(sizeof(T) * L) Pack {
    T v[L];
};
template <typename T, int L> __device__ __forceinline__ Pack<T, L> ldp(const T *p) {
    return *reinterpret_cast<const Pack<T, L> *>(p);
}
template <typename T, int L> __device__ __forceinline__ void stp(T *p, const Pack<T, L> &x) {
    *reinterpret_cast<Pack<T, L> *>(p) = x;
}
// six consecutive table entries (rows of [..][6] tables are 8-byte aligned
// for 4-byte types and 16-byte aligned for 8-byte types)
template <typename T> __device__ __forceinline__ void ld6(const T *p, T out[6]) {
    const Pack<T, 2> a = ldp<T, 2>(p), b = ldp<T, 2>(p + 2), c = ldp<T, 2>(p + 4);
    out[0] = a.v[0]; out[1] = a.v[1]; out[2] = b.v[0]; out[3] = b.v[1]; out[4] = c.v[0]; out[5] = c.v[1];
}

// a * b + c with one rounding.  The library is built without FMA contraction,
// so every fused operation is written out and is the same in every template
// instance (the results do not depend on the launch shape).
__device__ __forceinline__ float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }

// x^y for x > 0 as exp(y log x) (the exponents here are fixed gas constants
// and x a pressure ratio near 1, so this stays within a few ulps of pow)
__device__ __forceinline__ double powpos(double x, double y) { return exp(y * log(x)); }
__device__ __forceinline__ float powpos(float x, float y) { return expf(y * logf(x)); }

template <typename R> __device__ __forceinline__ const R *u_prev_ptr(const StageArgs &a) {
    if constexpr (sizeof(R) == 8) return a.u_s;
    else return a.u32_s;
}

// Lane decomposition: L values of (k, m) starting at km0.
template <int L, bool M1> struct Vals {
    int k0, mm0;
    int k[L];
    __device__ __forceinline__ Vals(int km0, int M) {
        k0 = M1 ? km0 : km0 / M;
        mm0 = km0 - k0 * M;
#pragma unroll
        for (int j = 0; j < L; j++) k[j] = M1 ? k0 + j : k0;
    }
};

// 2-D field (surface pressure, depth) of the L values at cell c
template <int L, bool M1> __device__ __forceinline__ void ld2d(const double *f, int c, int M, int mm0, double out[L]) {
    if constexpr (M1) {
        const double s = f[c];
#pragma unroll
        for (int j = 0; j < L; j++) out[j] = s;
    } else {
        const Pack<double, L> s = ldp<double, L>(f + (long)c * M + mm0);
#pragma unroll
        for (int j = 0; j < L; j++) out[j] = s.v[j];
    }
}

// layer mass from surface pressure (HDC/NDC) or depth (SW)
template <int MODEL> __device__ __forceinline__ double lmass(double dsg, double ps, double ptop) {
    if constexpr (MODEL == MODEL_SW) return ps;
    else return dsg * (ps - ptop);
}

// interface field X[N][K+1][M] at interface k + kk_off of the L values
template <int L, bool M1>
__device__ __forceinline__ void ld_iface(const double *X, long cbase, const Vals<L, M1> &v, int M, int kk_off,
                                         double out[L]) {
    if constexpr (M1) {
#pragma unroll
        for (int j = 0; j < L; j++) out[j] = X[cbase + v.k[j] + kk_off];
    } else {
        const Pack<double, L> p = ldp<double, L>(X + cbase + (long)(v.k0 + kk_off) * M + v.mm0);
#pragma unroll
        for (int j = 0; j < L; j++) out[j] = p.v[j];
    }
}
template <int L, bool M1>
__device__ __forceinline__ void st_iface(double *X, long cbase, const Vals<L, M1> &v, int M, int kk_off,
                                         const double in[L]) {
    if constexpr (M1) {
#pragma unroll
        for (int j = 0; j < L; j++) X[cbase + v.k[j] + kk_off] = in[j];
    } else {
        Pack<double, L> p;
#pragma unroll
        for (int j = 0; j < L; j++) p.v[j] = in[j];
        stp<double, L>(X + cbase + (long)(v.k0 + kk_off) * M + v.mm0, p);
    }
}

// theta of the previous stage at cell c, values starting at km0 (R precision)
template <int MODEL, typename R, int L>
__device__ __forceinline__ void theta_prev(const StageArgs &a, int c, long KM, unsigned km0, const double dsg[L],
                                           const double psc[L], R out[L]) {
    if constexpr (sizeof(R) == 8) {
        const Pack<double, L> T = ldp<double, L>(a.Th_s + (long)c * KM + km0);
#pragma unroll
        for (int j = 0; j < L; j++) out[j] = T.v[j] / lmass<MODEL>(dsg[j], psc[j], a.ptop);
    } else {
        const Pack<float, L> T = ldp<float, L>(a.th32_s + (long)c * KM + km0);
#pragma unroll
        for (int j = 0; j < L; j++) out[j] = T.v[j];
    }
}

// LDS of a column kernel's own column work (scans, column solve), in bytes;
// the staged tables follow it
__host__ __device__ inline size_t col_lds_bytes(int model, int which, int cpb, int K, int M) {
    const size_t KM = (size_t)K * M;
    size_t b = 0;
    // cell_a: D [cpb][KM], the NH interface mass flux [cpb][(K+1) M] and the
    // second buffer of the column scan [cpb][KM]
    if (which == KERNEL_CELL_A)
        b = cpb * KM * 8 + (model == MODEL_NDC ? cpb * (K + 1) * (size_t)M * 8 : 0) + cpb * KM * 8;
    if (which == KERNEL_CELL_B && model != MODEL_SW)
        // NDC: the column solve's arrays; HDC: alpha dpi, and for M > 1 the scan's second buffer
        b = model == MODEL_NDC ? cpb * (10 * KM + (K + 1) * (size_t)M) * 8 : (M > 1 ? 2 : 1) * cpb * KM * 8;
    return coltab_round(b);
}

// Pointers to the staged tables of a column work-group
template <typename R> struct ColTab {
    int *ce, *cn, *cv;
    double *ps, *psn, *dps;
    double *div64;           // cell_a: [cpb][6]
    R *div, *gk, *ke, *hs, *tk, *hd;
    __device__ ColTab(char *base, int model, int which, int cpb, int M) {
        const ColTabLayout l = coltab_layout(model, which, cpb, M, (int)sizeof(R));
        ce = (int *)(base + l.ce);
        cn = (int *)(base + l.cn);
        cv = (int *)(base + l.cv);
        ps = (double *)(base + l.ps);
        psn = (double *)(base + l.psn);
        dps = (double *)(base + l.dps);
        char *r = base + l.r;
        div64 = (double *)r;
        div = (R *)r;
        hd = (R *)(base + l.hd);
        if (which == KERNEL_CELL_A) {
            ke = (R *)(r + (size_t)cpb * 48);
            hs = ke + (size_t)cpb * 6;
            gk = tk = nullptr;
        } else {
            gk = div + (size_t)cpb * 6;
            tk = gk + (size_t)cpb * 6;
            ke = tk + (size_t)cpb * 36;
            hs = nullptr;
        }
    }
};

// Load the tables of the work-group's columns [i0, i0 + ncol) into LDS with
// all its threads (contiguous rows; the neighbours' surface pressures through
// c_nbr), then synchronise.
// (UNI: a uniform-cell work-group reads its tables with scalar loads, so only
// the surface pressures, which differ between members, are staged.)
template <int WHICH, int MODEL, typename R, bool M1, bool UNI = false>
__device__ __forceinline__ void stage_columns(const StageArgs &a, const ColTab<R> &t, int nthr) {
    const DevMesh &m = a.mesh;
    const int M = M1 ? 1 : a.M;
    const int tid = threadIdx.x;
    const long i0 = (long)xcd_block() * a.cpb;
    const int ncol = (int)((long)m.N - i0 < (long)a.cpb ? (long)m.N - i0 : (long)a.cpb);
    constexpr bool CA = WHICH == KERNEL_CELL_A, SW = MODEL == MODEL_SW;
    constexpr int VW = 16 / (int)sizeof(R);          // R values per 16-byte vector
    // vectors (pairs for the [.][6] and [.][18] tables) and scalars to move
    const int v6 = ncol * 3, v18 = ncol * 9, v36 = ncol * 36 / VW, v48 = ncol * 48 / VW;
    const int nM = ncol * M, nps = ncol * 7 * M;
    int nmax = v6 > nps ? v6 : nps;
    if (CA && !SW && v18 > nmax) nmax = v18;
    if (!CA && v36 > nmax) nmax = v36;
    if (!CA && !SW && v48 > nmax) nmax = v48;
    if constexpr (UNI) nmax = nps;   // >= nM
    // One pass moves one vector of every table per thread, branch-free: a
    // thread past the end of a table re-reads and re-writes its last vector
    // (the same value), so no load sits under a condition (the compiler would
    // sink it to its store and wait there) and the work-group waits for
    // memory about twice per pass -- a neighbour's pressure needs its index
    // first -- instead of once per table.  At the usual shapes there is one
    // pass: a column has K M / L >= 12 lanes.
    for (int x = tid; x < nmax; x += nthr) {
        const int xp = x < nps ? x : nps - 1;
        const int pc = xp / (7 * M), pr = xp - pc * 7 * M;
        const int psl = pr / M, pmm = pr - psl * M;
        const int nbr = m.c_nbr[(i0 + pc) * kCellSlots + (psl > 0 ? psl - 1 : 0)];
        if constexpr (UNI) {
            if constexpr (!CA && !SW) {
                const int xm = x < nM ? x : nM - 1;
                const double pn = a.ps_n[i0 * M + xm], dp = a.dps[i0 * M + xm];
                t.psn[xm] = pn;
                t.dps[xm] = dp;
            }
            t.ps[xp] = a.ps_s[(psl == 0 ? i0 + pc : (long)nbr) * M + pmm];
            continue;
        }
        const int x6 = x < v6 ? x : v6 - 1;
        const long o6 = i0 * kCellSlots + 2 * (long)x6;
        const Pack<int, 2> e2 = ldp<int, 2>(m.c_edge + o6);
        const Pack<int, 2> n2 = ldp<int, 2>(m.c_nbr + o6);
        if constexpr (CA) {
            const Pack<double, 2> d64 = ldp<double, 2>(m.c_div + o6);
            const Pack<R, 2> k2 = ldp<R, 2>(pick<R>(m.c_ke, m.c_ke32) + o6);
            if constexpr (!SW) {
                const int x18 = x < v18 ? x : v18 - 1;
                const Pack<R, 2> h2 = ldp<R, 2>(pick<R>(m.c_hess, m.c_hess32) + i0 * 3 * kCellSlots + 2 * (long)x18);
                stp<R, 2>(t.hs + 2 * x18, h2);
            }
            stp<double, 2>(t.div64 + 2 * x6, d64);
            stp<R, 2>(t.ke + 2 * x6, k2);
        } else {
            const Pack<int, 2> c2 = ldp<int, 2>(m.c_vert + o6);
            const Pack<R, 2> d2 = ldp<R, 2>(pick<R>(m.c_div, m.c_div32) + o6);
            const Pack<R, 2> g2 = ldp<R, 2>(pick<R>(m.c_gk, m.c_gk32) + o6);
            const int x36 = x < v36 ? x : v36 - 1;
            const Pack<R, VW> t4 = ldp<R, VW>(pick<R>(m.c_tk, m.c_tk32) + i0 * 36 + (long)VW * x36);
            if constexpr (!SW) {
                const int x48 = x < v48 ? x : v48 - 1;
                const Pack<R, VW> hd4 = ldp<R, VW>(pick<R>(m.c_hd, m.c_hd32) + i0 * 48 + (long)VW * x48);
                const int xm = x < nM ? x : nM - 1;
                const double pn = a.ps_n[i0 * M + xm], dp = a.dps[i0 * M + xm];
                stp<R, VW>(t.hd + VW * x48, hd4);
                t.psn[xm] = pn;
                t.dps[xm] = dp;
            }
            const Pack<R, 2> k2 = ldp<R, 2>(pick<R>(m.c_ke, m.c_ke32) + o6);
            stp<int, 2>(t.cv + 2 * x6, c2);
            stp<R, 2>(t.div + 2 * x6, d2);
            stp<R, 2>(t.gk + 2 * x6, g2);
            stp<R, 2>(t.ke + 2 * x6, k2);
            stp<R, VW>(t.tk + VW * x36, t4);
        }
        const double pv = a.ps_s[(psl == 0 ? i0 + pc : (long)nbr) * M + pmm];
        stp<int, 2>(t.ce + 2 * x6, e2);
        stp<int, 2>(t.cn + 2 * x6, n2);
        t.ps[xp] = pv;
    }
    __syncthreads();
}

// 2-D field of the L values from a staged row [M]
template <int L, bool M1> __device__ __forceinline__ void ld2d_s(const double *row, int mm0, double out[L]) {
    if constexpr (M1) {
        const double s = row[0];
#pragma unroll
        for (int j = 0; j < L; j++) out[j] = s;
    } else {
        const Pack<double, L> s = ldp<double, L>(row + mm0);
#pragma unroll
        for (int j = 0; j < L; j++) out[j] = s.v[j];
    }
}

// Slots of a column kernel's stencil loop per basic block: the gathers of a
// group are issued together and waited for once.  More slots per group means
// fewer memory round trips but more live registers; the sizes are the fastest
// measured on MI355X (G6 x 30).
template <int WHICH, typename R> constexpr int slot_group() {
    if constexpr (WHICH == KERNEL_CELL_A) return sizeof(R) == 8 ? 2 : 3;
    else return sizeof(R) == 8 ? 1 : 2;
}

// The FP32 policies (except the boxed variant, which forms the vertical
// advection in FP64) give the vertical mass flux's advective users, cell_b's
// vertical theta flux and edge's vertical advection of u, an FP32 copy of it
// written by cell_a: half the bytes and loads of the FP64 flux, which then
// is stored only for the tracer mass-flux accumulation.
template <typename R, int VAR> constexpr bool mdot32_used() { return sizeof(R) == 4 && VAR != VAR_BOX; }

// Where the kinetic energy K_i of a cell is formed.  Both column kernels load
// the cell's six edge velocities; in the FP32 policies cell_b forms K itself
// (saving cell_a's store and cell_b's load of K); in FP64 the four extra
// registers would cost cell_b a wave per SIMD, so cell_a forms and stores it;
// the boxed variant forms it in FP64 in cell_a.  Same sum either way.
template <typename R, int VAR> constexpr bool ke_in_cell_b() { return sizeof(R) == 4 && VAR != VAR_BOX; }

// column-kernel lane setup: work-group = cpb cells x (K*M/L) lanes
struct ColLane {
    int lc, km0, i;
    bool valid;
};
template <int L, bool UNI = false> __device__ __forceinline__ ColLane col_lane(const StageArgs &a, int KM) {
    ColLane c;
    if constexpr (UNI) {
        // one cell per work-group (of exactly K M / L lanes): the cell, and so
        // every value of its stencil tables, is the same in all lanes of a wave
        c.lc = 0;
        c.km0 = (int)threadIdx.x * L;
        c.i = (int)xcd_block();
        c.valid = c.i < a.mesh.N;
        return c;
    }
    const int lanes = KM / L;
    const int tid = threadIdx.x;
    c.lc = tid / lanes;
    c.km0 = (tid - c.lc * lanes) * L;
    c.i = (int)xcd_block() * a.cpb + c.lc;
    c.valid = (c.lc < a.cpb) && (c.i < a.mesh.N);
    return c;
}

// Sequential sum over LDS with the loads issued four at a time (the adds keep
// their order): s0 + sum over q = q_hi, q_hi-1, ..., q_lo+1, in precision T.
template <typename T>
__device__ __forceinline__ T lds_sum_down(const double *p, int stride, int q_hi, int q_lo, T s0) {
    T s = s0;
    int q = q_hi;
    for (; q - 4 >= q_lo; q -= 4) {
        const T a0 = (T)p[q * stride], a1 = (T)p[(q - 1) * stride], a2 = (T)p[(q - 2) * stride], a3 = (T)p[(q - 3) * stride];
        s += a0;
        s += a1;
        s += a2;
        s += a3;
    }
    for (; q > q_lo; q--) s += (T)p[q * stride];
    return s;
}

// ---------------------------------------------------------------------------
// cell_a
// ---------------------------------------------------------------------------
// Minimum waves per SIMD asked of the register allocator for a column
// kernel instance (1: no constraint).  The mixed-policy non-hydrostatic
// cell_a with two values per lane lands two registers above the four-wave
// boundary otherwise (measured 5% faster with the hint at G8 x 60).
template <int WHICH, int MODEL, typename R, int L> constexpr int col_waves() {
    if constexpr (WHICH == KERNEL_CELL_A && MODEL == MODEL_NDC && sizeof(R) == 4 && L == 2) return 4;
    return 1;
}

template <int MODEL, typename R, int L, bool M1, int VAR, bool UNI>
__global__ void __launch_bounds__(kColumnThreads)
__attribute__((amdgpu_waves_per_eu(col_waves<KERNEL_CELL_A, MODEL, R, L>())))
k_cell_a(StageArgs a) {
    // mixed-policy variants: the boxed kinetic energy and the FP64 mass flux
    // read the FP64 velocity instead of its FP32 shadow
    constexpr bool U64 = VAR == VAR_BOX || VAR == VAR_DBL_MASS;
    constexpr bool MDOT32 = mdot32_used<R, VAR>();
    extern __shared__ double lds[];
    const DevMesh &m = a.mesh;
    const int K = a.K, M = M1 ? 1 : a.M, KM = K * M;
    const ColLane cl = col_lane<L, UNI>(a, KM);
    const int i = cl.i, lc = cl.lc;
    const unsigned km0 = (unsigned)cl.km0;   // unsigned lane offset in a row (see k_cell_b)
    const Vals<L, M1> v((int)km0, M);
    double *sD = lds;                        // [cpb][KM]
    double *sMd = lds + a.cpb * KM;          // [cpb][(K+1) M]  (NDC)
    const ColTab<R> tb((char *)lds + col_lds_bytes(MODEL, KERNEL_CELL_A, a.cpb, K, a.M), MODEL, KERNEL_CELL_A, a.cpb, M);
    stage_columns<KERNEL_CELL_A, MODEL, R, M1, UNI>(a, tb, a.cpb * (KM / L));
    const long r6 = (long)i * kCellSlots;   // the cell's row of the [N][6] tables (scalar loads, UNI)
    const double *cps = tb.ps + (long)lc * 7 * M;   // ps_s of this cell, then of its neighbours

    double dsg[L], psi[L], dpi_i[L], D[L], sgb[L], ke64[L];
    float Df[L];   // literal FP32 divergence
    R ke[L], Fs[kCellSlots][L] = {};
    R h0[L], h1[L], h2[L], th_i[L];
    int ce[6], cn[6];
    if (cl.valid) {
#pragma unroll
        for (int j = 0; j < L; j++) sgb[j] = a.sig[v.k[j] + 1];   // read before the barrier
        ld2d_s<L, M1>(cps, v.mm0, psi);
#pragma unroll
        for (int j = 0; j < L; j++) {
            dsg[j] = (MODEL == MODEL_SW) ? 1.0 : a.dsig[v.k[j]];
            dpi_i[j] = lmass<MODEL>(dsg[j], psi[j], a.ptop);
            ke[j] = 0;
            D[j] = 0.0;
            Df[j] = 0.0f;
            ke64[j] = 0.0;
            h0[j] = h1[j] = h2[j] = 0;
        }
        double cdiv[6];
        R cke[6], ch0[6], ch1[6], ch2[6];
        if constexpr (UNI) {
            sld6<int>(m.c_edge, r6, ce);
            sld6<int>(m.c_nbr, r6, cn);
            sld6<double>(m.c_div, r6, cdiv);
            if constexpr (!ke_in_cell_b<R, VAR>()) sld6<R>(pick<R>(m.c_ke, m.c_ke32), r6, cke);
        } else {
            ld6<int>(tb.ce + lc * kCellSlots, ce);
            ld6<int>(tb.cn + lc * kCellSlots, cn);
            ld6<double>(tb.div64 + lc * kCellSlots, cdiv);
            if constexpr (!ke_in_cell_b<R, VAR>()) ld6<R>(tb.ke + lc * kCellSlots, cke);
        }
        double cked[6];   // FP64 kinetic-energy weights of the boxed variant
        if constexpr (VAR == VAR_BOX) ld6<double>(m.c_ke + (long)i * kCellSlots, cked);
        if constexpr (MODEL != MODEL_SW) {
            if constexpr (UNI) {
                const R *ch = pick<R>(m.c_hess, m.c_hess32);
                sld6<R>(ch, 3 * r6, ch0);
                sld6<R>(ch, 3 * r6 + kCellSlots, ch1);
                sld6<R>(ch, 3 * r6 + 2 * kCellSlots, ch2);
            } else {
                const R *ch = tb.hs + lc * 3 * kCellSlots;
                ld6<R>(ch, ch0);
                ld6<R>(ch + kCellSlots, ch1);
                ld6<R>(ch + 2 * kCellSlots, ch2);
            }
            theta_prev<MODEL, R, L>(a, i, KM, km0, dsg, psi, th_i);
        }
        const R *us = u_prev_ptr<R>(a);
#pragma unroll
        for (int s = 0; s < kCellSlots; s++) {
            // slot_group() slots per basic block (see k_cell_b); the pad slot
            // of a pentagon reads edge 0 and itself, with zero weights and flux
            if (s % slot_group<KERNEL_CELL_A, R>() == 0 && ce[s] < 0) continue;   // slots 0..4 always exist
            const bool pad = ce[s] < 0;
            const int e = pad ? 0 : ce[s];
            const int nb = cn[s];
            double psn[L];
            ld2d_s<L, M1>(cps + (1 + s) * M, v.mm0, psn);
            R ur[L];
            double ud[L];
            if constexpr (U64) {
                const Pack<double, L> u = ldp<double, L>(a.u_s + (long)e * KM + km0);
#pragma unroll
                for (int j = 0; j < L; j++) {
                    ud[j] = u.v[j];
                    ur[j] = (R)u.v[j];   // the FP32 shadow's value
                }
            } else {
                const Pack<R, L> u = ldp<R, L>(us + (long)e * KM + km0);
#pragma unroll
                for (int j = 0; j < L; j++) ur[j] = u.v[j];
            }
#pragma unroll
            for (int j = 0; j < L; j++) {
                const double dpe = 0.5 * (dpi_i[j] + lmass<MODEL>(dsg[j], psn[j], a.ptop));
                if constexpr (VAR == VAR_DBL_MASS) {
                    // continuity in FP64; the advective users take the flux rounded
                    const double f64 = pad ? 0.0 : dpe * ud[j];
                    Fs[s][j] = (R)f64;
                    D[j] += cdiv[s] * f64;
                } else {
                    R f;
                    if constexpr (sizeof(R) == 8) f = dpe * ur[j];
                    else f = (float)dpe * ur[j];
                    Fs[s][j] = pad ? (R)0 : f;
                    if constexpr (VAR == VAR_F32_DIV) Df[j] += (float)cdiv[s] * (float)Fs[s][j];
                    else if constexpr (sizeof(R) == 8) D[j] += cdiv[s] * Fs[s][j];
                    else D[j] += cdiv[s] * (double)Fs[s][j];
                }
                if constexpr (VAR == VAR_BOX) ke64[j] += cked[s] * ud[j] * ud[j];
                else if constexpr (!ke_in_cell_b<R, VAR>()) ke[j] += cke[s] * ur[j] * ur[j];
            }
            if constexpr (MODEL != MODEL_SW) {
                R th_n[L];
                theta_prev<MODEL, R, L>(a, nb, KM, km0, dsg, psn, th_n);
#pragma unroll
                for (int j = 0; j < L; j++) {
                    const R dth = th_n[j] - th_i[j];
                    h0[j] += ch0[s] * dth;
                    h1[j] += ch1[s] * dth;
                    h2[j] += ch2[s] * dth;
                }
            }
        }
        if constexpr (VAR == VAR_F32_DIV) {
#pragma unroll
            for (int j = 0; j < L; j++) D[j] = (double)Df[j];
        }
        if constexpr (VAR == VAR_BOX) {
            Pack<double, L> kp;
#pragma unroll
            for (int j = 0; j < L; j++) kp.v[j] = ke64[j];
            stp<double, L>((double *)a.ke + (long)i * KM + km0, kp);
        } else if constexpr (!ke_in_cell_b<R, VAR>()) {
            Pack<R, L> kp;
#pragma unroll
            for (int j = 0; j < L; j++) kp.v[j] = ke[j];
            stp<R, L>(a.ke_out<R>() + (long)i * KM + km0, kp);
        }
    }

    if constexpr (MODEL == MODEL_SW) {
        if (cl.valid) {
            // h^(s) = h^n - dt_s D  (forward part of the stage)
            double hn[L];
            ld2d<L, M1>(a.ps_n, i, M, v.mm0, hn);
            Pack<double, L> ho;
#pragma unroll
            for (int j = 0; j < L; j++) ho.v[j] = hn[j] + a.dts * (-D[j]);
            stp<double, L>(a.ps_o + (long)i * M + v.mm0, ho);
        }
        return;
    } else {
        // ---- column mass tendency and vertical mass flux (LDS scan) ----
        if (cl.valid) {
#pragma unroll
            for (int j = 0; j < L; j++) sD[lc * KM + km0 + j] = D[j];
        }
        __syncthreads();
        // The prefix sums over k of each column (and member) come from a
        // parallel scan in LDS (Hillis-Steele, double buffered, ceil(log2 K)
        // steps: after the step with distance d each entry holds the sum of the
        // 2d entries ending at it), far fewer LDS reads than a sequential sum
        // per lane.  The sums depend on k only, not on the launch shape.
        const double *scan = sD;
        {
            double *src = sD, *dst = sD + a.cpb * KM + (MODEL == MODEL_NDC ? a.cpb * (K + 1) * M : 0);
            for (int d = 1; d < K; d *= 2) {
                if (cl.valid) {
#pragma unroll
                    for (int j = 0; j < L; j++) {
                        const int o = lc * KM + v.k[j] * M + v.mm0 + (M1 ? 0 : j);
                        const double lo = src[o - (v.k[j] >= d ? d * M : 0)];   // clamped: unused below d
                        dst[o] = v.k[j] >= d ? src[o] + lo : src[o];
                    }
                }
                __syncthreads();
                double *tmp = src;
                src = dst;
                dst = tmp;
            }
            scan = src;
        }
        double mdot_b[L];
        if (cl.valid) {
            const long K1M = (long)(K + 1) * M;
            // FP32 policies: the FP32 copy for the advective users, and the FP64
            // flux only where the tracer accumulation reads it
            const bool st64 = !MDOT32 || a.mdot64;
            double dps[L];
#pragma unroll
            for (int j = 0; j < L; j++) {
                const int mm = v.mm0 + (M1 ? 0 : j);
                dps[j] = -scan[lc * KM + (K - 1) * M + mm];
                const double acc = scan[lc * KM + v.k[j] * M + mm];
                mdot_b[j] = (v.k[j] == K - 1) ? 0.0 : -acc - sgb[j] * dps[j];
            }
            if constexpr (M1) {
#pragma unroll
                for (int j = 0; j < L; j++) {
                    if (st64) a.mdot[(long)i * K1M + v.k[j] + 1] = mdot_b[j];
                    if constexpr (MDOT32) a.mdot32[(long)i * K1M + v.k[j] + 1] = (float)mdot_b[j];
                }
                if (v.k0 == 0) {
                    if (st64) a.mdot[(long)i * K1M] = 0.0;
                    if constexpr (MDOT32) a.mdot32[(long)i * K1M] = 0.0f;
                    a.dps[i] = dps[0];
                }
            } else {
                // the lane's L members of one interface are consecutive: one
                // vector store per array
                Pack<double, L> m64, z64, dp;
                Pack<float, L> m32, z32;
#pragma unroll
                for (int j = 0; j < L; j++) {
                    m64.v[j] = mdot_b[j];
                    m32.v[j] = (float)mdot_b[j];
                    z64.v[j] = 0.0;
                    z32.v[j] = 0.0f;
                    dp.v[j] = dps[j];
                }
                const long o = (long)i * K1M + (long)(v.k0 + 1) * M + v.mm0;
                if (st64) stp<double, L>(a.mdot + o, m64);
                if constexpr (MDOT32) stp<float, L>(a.mdot32 + o, m32);
                if (v.k0 == 0) {
                    if (st64) stp<double, L>(a.mdot + (long)i * K1M + v.mm0, z64);
                    if constexpr (MDOT32) stp<float, L>(a.mdot32 + (long)i * K1M + v.mm0, z32);
                    stp<double, L>(a.dps + (long)i * M + v.mm0, dp);
                }
            }
            // ---- second derivatives of theta ----
            Pack<R, L> p0, p1, p2;
#pragma unroll
            for (int j = 0; j < L; j++) {
                p0.v[j] = h0[j];
                p1.v[j] = h1[j];
                p2.v[j] = h2[j];
            }
            R *H = a.hth_out<R>() + (long)i * 3 * KM + km0;
            stp<R, L>(H, p0);
            stp<R, L>(H + KM, p1);
            stp<R, L>(H + 2 * KM, p2);
        }

        if constexpr (MODEL == MODEL_NDC) {
            // ---- explicit advective step of w and phi at interface k ----
            const int K1 = K + 1;
            if (cl.valid) {
#pragma unroll
                for (int j = 0; j < L; j++) {
                    const int mm = v.mm0 + (M1 ? 0 : j);
                    sMd[lc * K1 * M + (v.k[j] + 1) * M + mm] = mdot_b[j];
                    if (v.k[j] == 0) sMd[lc * K1 * M + mm] = 0.0;
                }
            }
            __syncthreads();
            if (cl.valid) {
                const long K1M = (long)K1 * M;
                const long cb = (long)i * K1M;
                const double *md = sMd + lc * K1 * M;
                // interface masses (half layers either side; half of layer 0 at the top)
                double dh[L];
#pragma unroll
                for (int j = 0; j < L; j++) {
                    // masses as factors, not branches (the top interface has no layer above)
                    const double dkm = (v.k[j] > 0 ? 1.0 : 0.0) * lmass<MODEL>(a.dsig[v.k[j] - (v.k[j] > 0)], psi[j], a.ptop);
                    dh[j] = 0.5 * (dkm + dpi_i[j]);
                }
                double wi[L], pi_[L];
                ld_iface<L, M1>(a.w_s, cb, v, M, 0, wi);
                ld_iface<L, M1>(a.phi_s, cb, v, M, 0, pi_);
                const R *us = u_prev_ptr<R>(a);
                R aw[L], ap[L], asf[L];
#pragma unroll
                for (int j = 0; j < L; j++) aw[j] = ap[j] = asf[j] = 0;
                // lanes holding the bottom layer also form the kinematic surface w
                // (g w_s = V.grad phi_s: the horizontal advection of phi at the
                // surface interface, the bottom layer's flux at half weight); over
                // a flat surface it is zero and the gathers are skipped
                const bool bottom = (M1 ? v.k0 + L - 1 : v.k0) >= K - 1 && *a.nh_terrain != 0;
                double pd[L];
                ld_iface<L, M1>(a.phi_s, cb, v, M, 1, pd);
                double cdiv[6];
                if constexpr (UNI) sld6<double>(m.c_div, r6, cdiv);
                else ld6<double>(tb.div64 + lc * kCellSlots, cdiv);
                // slots grouped per basic block and no load under a condition,
                // as in the horizontal part above (pad slot: edge 0, itself,
                // zero flux and weight; the layer above the top: clamped index)
                const bool up = v.k0 > 0;
                const double dsu = a.dsig[v.k0 - (int)up];
                const R mup = up ? (R)1 : (R)0;   // the layer above: a factor, not a branch
#pragma unroll
                for (int s = 0; s < kCellSlots; s++) {
                    if (s % slot_group<KERNEL_CELL_A, R>() == 0 && ce[s] < 0) continue;   // never taken
                    const int e = ce[s] < 0 ? 0 : ce[s];
                    const int nb = cn[s];
                    double psn[L];
                    ld2d_s<L, M1>(cps + (1 + s) * M, v.mm0, psn);
                    // mass flux of the layer above each value (for the interface average)
                    R Fm[L];
                    if constexpr (M1) {
#pragma unroll
                        for (int j = 1; j < L; j++) Fm[j] = Fs[s][j - 1];
                        const double d1 = lmass<MODEL>(dsu, psi[0], a.ptop);
                        const double d2 = lmass<MODEL>(dsu, psn[0], a.ptop);
                        const R um = us[(long)e * KM + km0 - (up ? 1 : 0)];
                        R f;
                        if constexpr (sizeof(R) == 8) f = 0.5 * (d1 + d2) * um;
                        else f = (float)(0.5 * (d1 + d2)) * um;
                        Fm[0] = mup * f;
                    } else {
                        const Pack<R, L> um = ldp<R, L>(us + (long)e * KM + km0 - (up ? M : 0));
#pragma unroll
                        for (int j = 0; j < L; j++) {
                            const double d1 = lmass<MODEL>(dsu, psi[j], a.ptop);
                            const double d2 = lmass<MODEL>(dsu, psn[j], a.ptop);
                            R f;
                            if constexpr (sizeof(R) == 8) f = 0.5 * (d1 + d2) * um.v[j];
                            else f = (float)(0.5 * (d1 + d2)) * um.v[j];
                            Fm[j] = mup * f;
                        }
                    }
                    double wn_[L], pn_[L];
                    ld_iface<L, M1>(a.w_s, (long)nb * K1M, v, M, 0, wn_);
                    ld_iface<L, M1>(a.phi_s, (long)nb * K1M, v, M, 0, pn_);
#pragma unroll
                    for (int j = 0; j < L; j++) {
                        const R Fh = (R)0.5 * (Fm[j] + Fs[s][j]);   // Fm = 0 at the top interface
                        const R c = (R)cdiv[s] * Fh * (R)0.5;
                        aw[j] += c * (R)(wn_[j] - wi[j]);
                        ap[j] += c * (R)(pn_[j] - pi_[j]);
                    }
                    if (bottom) {
                        double pnK[L];
                        ld_iface<L, M1>(a.phi_s, (long)nb * K1M, v, M, 1, pnK);
#pragma unroll
                        for (int j = 0; j < L; j++) {
                            const R c = (R)cdiv[s] * ((R)0.5 * Fs[s][j]) * (R)0.5;
                            asf[j] += c * (R)(pnK[j] - pd[j]);
                        }
                    }
                }
                // surface w of the lanes at layer K-1 (1/(half the bottom layer's mass))
                double wsf[L];
#pragma unroll
                for (int j = 0; j < L; j++)
                    wsf[j] = (double)(asf[j] * (R)(1.0 / (0.5 * dpi_i[j]))) / a.grav;
                double wu[L], wd[L], pu[L], wn0[L], pn0[L], ws_[L], ps_[L];
                ld_iface<L, M1>(a.w_n, cb, v, M, 0, wn0);
                ld_iface<L, M1>(a.phi_n, cb, v, M, 0, pn0);
                ld_iface<L, M1>(a.w_s, cb, v, M, 1, wd);
#pragma unroll
                for (int j = 0; j < L; j++)
                    if (v.k[j] == K - 1) wd[j] = wsf[j];   // the surface: this stage's kinematic w
                // the interface above each value (none above the top interface)
                if constexpr (M1) {
#pragma unroll
                    for (int j = 0; j < L; j++) {
                        const int kq = v.k[j] - (v.k[j] >= 1);   // clamped; unused at the top
                        wu[j] = a.w_s[cb + kq];
                        pu[j] = a.phi_s[cb + kq];
                    }
                } else {
                    ld_iface<L, M1>(a.w_s, cb, v, M, -(int)up, wu);   // unused at the top
                    ld_iface<L, M1>(a.phi_s, cb, v, M, -(int)up, pu);
                }
#pragma unroll
                for (int j = 0; j < L; j++) {
                    const int kk = v.k[j], mm = v.mm0 + (M1 ? 0 : j);
                    const R inv_dh = (R)(1.0 / dh[j]);
                    R vw = 0, vp = 0;
                    {
                        const R fu = kk >= 1 ? (R)1 : (R)0;   // no interface above the top one
                        const R ml = (R)(0.5 * (md[(kk - (kk >= 1)) * M + mm] + md[kk * M + mm]));
                        vw += fu * (ml * (R)(wi[j] - wu[j]));
                        vp += fu * (ml * (R)(pi_[j] - pu[j]));
                    }
                    {
                        const R ml = (R)(0.5 * (md[kk * M + mm] + md[(kk + 1) * M + mm]));
                        vw += ml * (R)(wd[j] - wi[j]);
                        vp += ml * (R)(pd[j] - pi_[j]);
                    }
                    const R advw = aw[j] * inv_dh + vw * (inv_dh * (R)0.5);
                    const R advp = ap[j] * inv_dh + vp * (inv_dh * (R)0.5);
                    ws_[j] = (kk == 0 ? 0.0 : 1.0) * (wn0[j] - a.dts * (double)advw);   // w = 0 at the lid
                    ps_[j] = pn0[j] - a.dts * (double)advp;
                }
                st_iface<L, M1>(a.wstar, cb, v, M, 0, ws_);
                st_iface<L, M1>(a.phistar, cb, v, M, 0, ps_);
                // surface interface: the kinematic w, phi fixed at phi_s
#pragma unroll
                for (int j = 0; j < L; j++) {
                    if (v.k[j] == K - 1) {
                        const int mm = v.mm0 + (M1 ? 0 : j);
                        a.wstar[cb + (long)K * M + mm] = wsf[j];
                        a.phistar[cb + (long)K * M + mm] = a.phi_n[cb + (long)K * M + mm];
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// vertex: vorticity, FP64 vertex mass, potential vorticity
// ---------------------------------------------------------------------------
// LDS of the vertex kernel: per vertex of the work-group its f, three kite
// weights, three curl weights, three edges and the three cells' surface
// pressures [3][M]; then dsig [K].  Doubles throughout (the curl weights and
// edge indices are exact in them).  Shapes whose vertices would not fit
// 64 KiB (a vertex of very few lanes in a large work-group) read their
// tables directly instead.
__host__ __device__ inline int vertex_stage_max(int flat_block, int lanes) { return flat_block / lanes + 2; }
__host__ __device__ inline size_t vertex_lds_bytes(int flat_block, int lanes, int K, int M) {
    return ((size_t)vertex_stage_max(flat_block, lanes) * (10 + 3 * (size_t)M) + (size_t)K) * 8;
}
constexpr size_t kVertexLdsMax = 65536;

// One vertex's constants: f, kite weights, curl weights, edges (as doubles).
__device__ __forceinline__ void vertex_row(const DevMesh &m, long vx, bool f32curl, double t[10]) {
    const Pack<int, 4> ve = ldp<int, 4>(m.v_edge + 4 * vx);
    const Pack<double, 2> k0 = ldp<double, 2>(m.v_kite + 4 * vx), k1 = ldp<double, 2>(m.v_kite + 4 * vx + 2);
    t[0] = m.v_f[vx];
    t[1] = k0.v[0]; t[2] = k0.v[1]; t[3] = k1.v[0];
    if (f32curl) {
        const Pack<float, 4> c = ldp<float, 4>(m.v_curl32 + 4 * vx);
        t[4] = (double)c.v[0]; t[5] = (double)c.v[1]; t[6] = (double)c.v[2];
    } else {
        const Pack<double, 2> c0 = ldp<double, 2>(m.v_curl + 4 * vx), c1 = ldp<double, 2>(m.v_curl + 4 * vx + 2);
        t[4] = c0.v[0]; t[5] = c0.v[1]; t[6] = c1.v[0];
    }
    t[7] = (double)ve.v[0]; t[8] = (double)ve.v[1]; t[9] = (double)ve.v[2];
}

template <int MODEL, typename R, int L, bool M1, int VAR, bool STAGED>
__global__ void __launch_bounds__(1024) k_vertex(StageArgs a) {
    // the all-FP32 variant forms the vertex mass and the potential vorticity in
    // FP32 (the paper keeps the vertex mass of zeta_p in FP64)
    constexpr bool S32 = VAR == VAR_SGL;
    using RM = typename std::conditional<S32, float, double>::type;
    extern __shared__ double vlds[];
    const DevMesh &m = a.mesh;
    const int K = a.K, M = M1 ? 1 : a.M, KM = K * M;
    const int lanes = KM / L;
    const long b0 = (long)xcd_block() * a.flat_block;
    const long nall = (long)m.V * lanes;
    const long idx = b0 + threadIdx.x;
    // The work-group's vertices share their tables and cells' surface
    // pressures among all K M / L lanes of each vertex: staged once in LDS,
    // so the lanes issue only their three velocity gathers.
    const int v0 = (int)(b0 / lanes);
    const int nvm = vertex_stage_max(a.flat_block, lanes);
    double *sT = vlds;                              // [nvm][10]: f, kite[3], curl[3], edge[3]
    double *sP = sT + (long)nvm * 10;               // [nvm][3][M]
    double *sD = sP + (long)nvm * 3 * M;            // [K]
    if constexpr (STAGED) {
        const long lastl = (b0 + a.flat_block < nall ? b0 + a.flat_block : nall) - 1;
        const int nv = (int)(lastl / lanes) - v0 + 1;
        const int nrow = nv * 3 * M;
        for (int x = threadIdx.x; x < nv + nrow + K; x += blockDim.x) {
            if (x < nv) {
                vertex_row(m, v0 + x, sizeof(R) == 4, sT + (long)x * 10);
            } else if (x < nv + nrow) {
                const int y = x - nv, vs = y / (3 * M), r = (y - vs * 3 * M) / M, mm = y - vs * 3 * M - r * M;
                const int c = m.v_cell[4 * (long)(v0 + vs) + r];
                sP[y] = a.ps_s[(long)c * M + mm];
            } else {
                sD[x - nv - nrow] = a.dsig[x - nv - nrow];
            }
        }
        __syncthreads();
    }
    if (idx >= nall) return;
    const int vx = (int)(idx / lanes);
    const int km0 = (int)(idx - (long)vx * lanes) * L;
    const Vals<L, M1> v(km0, M);
    double trow[10];
    const double *t;
    Pack<int, 4> vc;
    if constexpr (STAGED) {
        t = sT + (long)(vx - v0) * 10;
    } else {
        vertex_row(m, vx, sizeof(R) == 4, trow);
        vc = ldp<int, 4>(m.v_cell + 4 * (long)vx);
        t = trow;
    }
    const RM kw[3] = {(RM)t[1], (RM)t[2], (RM)t[3]};
    const R cw[3] = {(R)t[4], (R)t[5], (R)t[6]};
    double dsg[L];
#pragma unroll
    for (int j = 0; j < L; j++) dsg[j] = (MODEL == MODEL_SW) ? 1.0 : STAGED ? sD[v.k[j]] : a.dsig[v.k[j]];
    R zeta[L];
    RM hv[L];
#pragma unroll
    for (int j = 0; j < L; j++) {
        zeta[j] = 0;
        hv[j] = 0;
    }
    const R *us = u_prev_ptr<R>(a);
#pragma unroll
    for (int r = 0; r < 3; r++) {
        const int e = (int)t[7 + r];
        const Pack<R, L> u = ldp<R, L>(us + (long)e * KM + km0);
        double ps[L];
        if constexpr (STAGED) ld2d_s<L, M1>(sP + ((long)(vx - v0) * 3 + r) * M, v.mm0, ps);
        else ld2d<L, M1>(a.ps_s, vc.v[r], M, v.mm0, ps);
#pragma unroll
        for (int j = 0; j < L; j++) {
            zeta[j] += cw[r] * u.v[j];
            hv[j] += kw[r] * (RM)lmass<MODEL>(dsg[j], ps[j], a.ptop);
        }
    }
    const double f = t[0];
    Pack<R, L> q;
#pragma unroll
    for (int j = 0; j < L; j++) {
        if constexpr (S32) q.v[j] = (zeta[j] + (float)f) / hv[j];
        else q.v[j] = (R)(((double)zeta[j] + f) / hv[j]);
    }
    stp<R, L>(a.qv_out<R>() + (long)vx * KM + km0, q);
}

// ---------------------------------------------------------------------------
// cell_b: Coriolis/KE shares, theta transport, mass/Theta update, column
// diagnostics or the NH column solve
// ---------------------------------------------------------------------------
template <int MODEL, typename R, int L, bool M1, int VAR, bool UNI>
__global__ void __launch_bounds__(kColumnThreads) k_cell_b(StageArgs a) {
    extern __shared__ double lds[];
    const DevMesh &m = a.mesh;
    const int K = a.K, M = M1 ? 1 : a.M, KM = K * M;
    const ColLane cl = col_lane<L, UNI>(a, KM);
    const int i = cl.i, lc = cl.lc;
    // the lane's offset in a row of K M values: unsigned, so that a row's
    // address (the same in every lane where the cell is) plus it is a
    // scalar-base-plus-vector-offset access
    const unsigned km0 = (unsigned)cl.km0;
    const Vals<L, M1> v((int)km0, M);
    const ColTab<R> tb((char *)lds + col_lds_bytes(MODEL, KERNEL_CELL_B, a.cpb, K, a.M), MODEL, KERNEL_CELL_B, a.cpb, M);
    stage_columns<KERNEL_CELL_B, MODEL, R, M1, UNI>(a, tb, a.cpb * (KM / L));
    const long r6 = (long)i * kCellSlots;   // the cell's row of the [N][6] tables (scalar loads, UNI)
    const double *cps = tb.ps + (long)lc * 7 * M;   // ps_s of this cell, then of its neighbours

    double Th_new[L], ps_new[L], dsg[L], sgt[L], sgb[L];
    if (cl.valid) {
        // sigma at the layer's interfaces for the column diagnostics: read
        // here, before the barriers, in the mixed policy (in FP64 the extra
        // live registers cost more than the late read)
        if constexpr (sizeof(R) == 4) {
#pragma unroll
            for (int j = 0; j < L; j++) {
                sgt[j] = a.sig[v.k[j]];
                sgb[j] = a.sig[v.k[j] + 1];
            }
        }
        double psi[L], dpi_i[L];
        ld2d_s<L, M1>(cps, v.mm0, psi);
#pragma unroll
        for (int j = 0; j < L; j++) {
            dsg[j] = (MODEL == MODEL_SW) ? 1.0 : a.dsig[v.k[j]];
            dpi_i[j] = lmass<MODEL>(dsg[j], psi[j], a.ptop);
        }
        int ce[6], cn[6], cv[6];
        R cdiv[6], cgk[6];
        if constexpr (UNI) {
            sld6<int>(m.c_edge, r6, ce);
            sld6<int>(m.c_nbr, r6, cn);
            sld6<int>(m.c_vert, r6, cv);
            sld6<R>(pick<R>(m.c_div, m.c_div32), r6, cdiv);
            sld6<R>(pick<R>(m.c_gk, m.c_gk32), r6, cgk);
        } else {
            ld6<int>(tb.ce + lc * kCellSlots, ce);
            ld6<int>(tb.cn + lc * kCellSlots, cn);
            ld6<int>(tb.cv + lc * kCellSlots, cv);
            ld6<R>(tb.div + lc * kCellSlots, cdiv);
            ld6<R>(tb.gk + lc * kCellSlots, cgk);
        }
        const R *us = u_prev_ptr<R>(a);
        const R *Hs = a.hth_in<R>();

        R th_i[L], Hi0[L], Hi1[L], Hi2[L];
        if constexpr (MODEL != MODEL_SW) {
            theta_prev<MODEL, R, L>(a, i, KM, km0, dsg, psi, th_i);
            const Pack<R, L> a0 = ldp<R, L>(Hs + (long)i * 3 * KM + km0);
            const Pack<R, L> a1 = ldp<R, L>(Hs + (long)i * 3 * KM + KM + km0);
            const Pack<R, L> a2 = ldp<R, L>(Hs + (long)i * 3 * KM + 2 * KM + km0);
#pragma unroll
            for (int j = 0; j < L; j++) {
                Hi0[j] = a0.v[j];
                Hi1[j] = a1.v[j];
                Hi2[j] = a2.v[j];
            }
        }
        // fluxes of the six edges, the theta flux divergence and the kinetic
        // energy K_i = sum (l d / 4 A) u^2 of the cell (Eq. 5)
        R Fs[kCellSlots][L] = {}, hdiv[L], ke[L];
#pragma unroll
        for (int j = 0; j < L; j++) hdiv[j] = ke[j] = 0;
#pragma unroll
        for (int s = 0; s < kCellSlots; s++) {
            // slot_group() slots per basic block: the gathers of a block are
            // issued together and waited for once; with no branch between
            // slots at all the compiler issues all six slots' gathers at once
            // and needs about twice the registers (measured slower).  The
            // branch is never taken (slots 0..4 exist in every cell); the pad
            // slot of a pentagon reads edge 0 and the cell itself, with zero
            // weights and flux.
            if (s % slot_group<KERNEL_CELL_B, R>() == 0 && ce[s] < 0) continue;
            const bool pad = ce[s] < 0;
            const int e = pad ? 0 : ce[s];
            const int nb = cn[s];
            double psn[L];
            ld2d_s<L, M1>(cps + (1 + s) * M, v.mm0, psn);
            const Pack<R, L> u = ldp<R, L>(us + (long)e * KM + km0);
            // kinetic-energy weight (zero on a pad slot)
            const R ck = UNI ? sld(pick<R>(m.c_ke, m.c_ke32), r6 + s) : tb.ke[lc * kCellSlots + s];
#pragma unroll
            for (int j = 0; j < L; j++) {
                const double dpe = 0.5 * (dpi_i[j] + lmass<MODEL>(dsg[j], psn[j], a.ptop));
                R f;
                if constexpr (sizeof(R) == 8) f = dpe * u.v[j];
                else f = (float)dpe * u.v[j];
                Fs[s][j] = pad ? (R)0 : f;
                if constexpr (ke_in_cell_b<R, VAR>()) ke[j] += ck * u.v[j] * u.v[j];
            }
            if constexpr (MODEL != MODEL_SW) {
                // Third-order upwind edge value: with the upwind weight 1 the two
                // second-derivative terms reduce to -d^2/6 times the second
                // derivative (along the edge) of the upwind cell alone.  Fs is the
                // flux along n_e (c1 -> c2), the same number from either cell.
                const bool c1 = cdiv[s] > (R)0;                 // i is c1 of e
                R th_n[L];
                theta_prev<MODEL, R, L>(a, nb, KM, km0, dsg, psn, th_n);
                // neighbour direction in i's frame, i's direction in the neighbour's, -d^2/6
                R hd[8];
                if constexpr (UNI) {
#pragma unroll
                    for (int q = 0; q < 8; q++) hd[q] = sld(pick<R>(m.c_hd, m.c_hd32), (r6 + s) * 8 + q);
                } else {
                    const R *p = tb.hd + (lc * kCellSlots + s) * 8;
#pragma unroll
                    for (int q = 0; q < 8; q += 2) {
                        const Pack<R, 2> x = ldp<R, 2>(p + q);
                        hd[q] = x.v[0];
                        hd[q + 1] = x.v[1];
                    }
                }
                const R *ds = hd, *dn = hd + 3;
                // (the neighbour's second derivatives are loaded whether or not it
                // is upwind: a load under a condition costs a wait where the paths join)
                const R *hb = Hs + (long)nb * 3 * KM;
                const Pack<R, L> b0 = ldp<R, L>(hb + km0), b1 = ldp<R, L>(hb + KM + km0), b2 = ldp<R, L>(hb + 2 * KM + km0);
                const R m2c = hd[6];
#pragma unroll
                for (int j = 0; j < L; j++) {
                    const bool up_i = (Fs[s][j] >= (R)0) == c1;
                    const R hi = fmar(Hi0[j], ds[0], fmar(Hi1[j], ds[1], Hi2[j] * ds[2]));
                    const R hn = fmar(b0.v[j], dn[0], fmar(b1.v[j], dn[1], b2.v[j] * dn[2]));
                    const R tv = fmar(m2c, up_i ? hi : hn, (R)0.5 * (th_i[j] + th_n[j]));
                    hdiv[j] = fmar(cdiv[s], Fs[s][j] * tv, hdiv[j]);
                }
            }
        }
        // ---- this cell's share of Coriolis - grad K on each of its edges (TRiSK) ----
        // With Q_s = q_v(s) + q_v(s+1) (twice the PV of edge s) the half sum
        //   sum_t w F_t (q_e(s) + q_e(t)) / 2 = Q_s sum_t w' F_t + sum_t w' F_t Q_t
        // with w' = w / 4 (the table holds w l_t / d_s already divided by 4).
        {
            R Q[kCellSlots][L], G[kCellSlots][L];
            {
                R QV[kCellSlots][L];
#pragma unroll
                for (int s = 0; s < kCellSlots; s++) {
                    const Pack<R, L> q = ldp<R, L>(a.qv_in<R>() + (long)cv[s] * KM + km0);
#pragma unroll
                    for (int j = 0; j < L; j++) QV[s][j] = q.v[j];
                }
#pragma unroll
                for (int s = 0; s < kCellSlots; s++)
#pragma unroll
                    for (int j = 0; j < L; j++) {
                        Q[s][j] = QV[s][j] + QV[(s + 1) % kCellSlots][j];
                        G[s][j] = Fs[s][j] * Q[s][j];
                    }
            }
            // (the boxed variant adds -grad K in FP64 on the edge instead)
            if constexpr (!ke_in_cell_b<R, VAR>() && VAR != VAR_BOX) {
                const Pack<R, L> kp = ldp<R, L>(a.ke_in<R>() + (long)i * KM + km0);
#pragma unroll
                for (int j = 0; j < L; j++) ke[j] = kp.v[j];
            }
            const R *tk = tb.tk + lc * kCellSlots * kCellSlots;
            R *qh = a.qh_out<R>();
#pragma unroll
            for (int s = 0; s < kCellSlots; s++) {
                const int e = ce[s];
                if (e < 0) continue;
                R w[6];
                if constexpr (UNI) sld6<R>(pick<R>(m.c_tk, m.c_tk32), (r6 + s) * kCellSlots, w);
                else ld6<R>(tk + s * kCellSlots, w);
                Pack<R, L> out;
#pragma unroll
                for (int j = 0; j < L; j++) {
                    const int s1 = (s + 1) % kCellSlots;
                    R A = w[s1] * Fs[s1][j], B = w[s1] * G[s1][j];
#pragma unroll
                    for (int t = 2; t < kCellSlots; t++) {
                        const int sp = (s + t) % kCellSlots;
                        A = fmar(w[sp], Fs[sp][j], A);
                        B = fmar(w[sp], G[sp][j], B);
                    }
                    if constexpr (VAR == VAR_BOX) out.v[j] = fmar(Q[s][j], A, B);
                    else out.v[j] = fmar(cgk[s], ke[j], fmar(Q[s][j], A, B));
                }
                const int side = (cdiv[s] > (R)0) ? 0 : 1;
                stp<R, L>(qh + ((long)e * 2 + side) * KM + km0, out);
            }
        }
        if constexpr (MODEL != MODEL_SW) {
            // vertical theta flux through the layer's interfaces (centred theta)
            const long K1M = (long)(K + 1) * M;
            const double *md = a.mdot + (long)i * K1M;
            // theta of the layers above and below: read from clamped indices
            // (the top and bottom values are not used), so no load is conditional
            R thu[L], thd[L];
            const bool has_up = v.k0 > 0;
            double vb[L];   // boxed variant: bottom minus top flux in FP64
            if constexpr (VAR == VAR_BOX) {
                double t64[L], tu[L], td[L];
                theta_prev<MODEL, double, L>(a, i, KM, km0, dsg, psi, t64);
                if constexpr (M1) {
                    const int kl = v.k[L - 1];
                    const bool has_dn = kl < K - 1;
                    const long ou = (long)i * KM + (has_up ? km0 - 1 : km0), od = (long)i * KM + (has_dn ? km0 + L : km0);
                    const double up = a.Th_s[ou] / lmass<MODEL>(a.dsig[has_up ? v.k0 - 1 : v.k0], psi[0], a.ptop);
                    const double dn = a.Th_s[od] / lmass<MODEL>(a.dsig[has_dn ? kl + 1 : kl], psi[0], a.ptop);
#pragma unroll
                    for (int j = 0; j < L; j++) {
                        tu[j] = j > 0 ? t64[j - 1] : up;
                        td[j] = j < L - 1 ? t64[j + 1] : dn;
                    }
                } else {
                    const bool has_dn = v.k0 < K - 1;
                    double du[L], dd[L];
#pragma unroll
                    for (int j = 0; j < L; j++) {
                        du[j] = a.dsig[has_up ? v.k0 - 1 : v.k0];
                        dd[j] = a.dsig[has_dn ? v.k0 + 1 : v.k0];
                    }
                    theta_prev<MODEL, double, L>(a, i, KM, has_up ? km0 - M : km0, du, psi, tu);
                    theta_prev<MODEL, double, L>(a, i, KM, has_dn ? km0 + M : km0, dd, psi, td);
                }
#pragma unroll
                for (int j = 0; j < L; j++) {
                    const int mm = v.mm0 + (M1 ? 0 : j);
                    const double mt = md[(long)v.k[j] * M + mm], mb = md[(long)(v.k[j] + 1) * M + mm];
                    const double top = (v.k[j] > 0 ? 1.0 : 0.0) * (mt * (0.5 * (tu[j] + t64[j])));
                    const double bot = (v.k[j] < K - 1 ? 1.0 : 0.0) * (mb * (0.5 * (t64[j] + td[j])));
                    vb[j] = bot - top;
                }
            } else if constexpr (M1) {
                const int kl = v.k[L - 1];
                const bool has_dn = kl < K - 1;
#pragma unroll
                for (int j = 0; j < L; j++) {
                    thu[j] = j > 0 ? th_i[j - 1] : (R)0;
                    thd[j] = j < L - 1 ? th_i[j + 1] : (R)0;
                }
                const long ou = (long)i * KM + (has_up ? km0 - 1 : km0), od = (long)i * KM + (has_dn ? km0 + L : km0);
                R up, dn;
                if constexpr (sizeof(R) == 8) {
                    up = a.Th_s[ou] / lmass<MODEL>(a.dsig[has_up ? v.k0 - 1 : v.k0], psi[0], a.ptop);
                    dn = a.Th_s[od] / lmass<MODEL>(a.dsig[has_dn ? kl + 1 : kl], psi[0], a.ptop);
                } else {
                    up = a.th32_s[ou];
                    dn = a.th32_s[od];
                }
                thu[0] = up;      // unused (multiplied by zero below) at the lid
                thd[L - 1] = dn;  // and at the surface
            } else {
                const bool has_dn = v.k0 < K - 1;
                double du[L], dd[L];
#pragma unroll
                for (int j = 0; j < L; j++) {
                    du[j] = a.dsig[has_up ? v.k0 - 1 : v.k0];
                    dd[j] = a.dsig[has_dn ? v.k0 + 1 : v.k0];
                }
                R tu[L], td[L];
                theta_prev<MODEL, R, L>(a, i, KM, has_up ? km0 - M : km0, du, psi, tu);
                theta_prev<MODEL, R, L>(a, i, KM, has_dn ? km0 + M : km0, dd, psi, td);
#pragma unroll
                for (int j = 0; j < L; j++) {
                    thu[j] = tu[j];
                    thd[j] = td[j];
                }
            }
            double dps_[L], psn_[L];
            ld2d_s<L, M1>(tb.dps + lc * M, v.mm0, dps_);
            ld2d_s<L, M1>(tb.psn + lc * M, v.mm0, psn_);
            const Pack<double, L> Thn = ldp<double, L>(a.Th_n + (long)i * KM + km0);
#pragma unroll
            for (int j = 0; j < L; j++) {
                const int mm = v.mm0 + (M1 ? 0 : j);
                // interfaces k and k + 1 always exist in mdot [K+1]; the flux
                // through the lid and the surface is zero
                R vd;
                if constexpr (VAR == VAR_BOX) {
                    vd = (R)vb[j];   // FP64 compute, one rounding as a tendency
                } else if constexpr (mdot32_used<R, VAR>()) {
                    const float *m32 = a.mdot32 + (long)i * K1M;
                    const R mt = m32[(long)v.k[j] * M + mm], mb = m32[(long)(v.k[j] + 1) * M + mm];
                    const R top = (v.k[j] > 0 ? (R)1 : (R)0) * (mt * ((R)0.5 * (thu[j] + th_i[j])));
                    const R bot = (v.k[j] < K - 1 ? (R)1 : (R)0) * (mb * ((R)0.5 * (th_i[j] + thd[j])));
                    vd = bot - top;
                } else {
                    const R mt = (R)md[(long)v.k[j] * M + mm], mb = (R)md[(long)(v.k[j] + 1) * M + mm];
                    const R top = (v.k[j] > 0 ? (R)1 : (R)0) * (mt * ((R)0.5 * (thu[j] + th_i[j])));
                    const R bot = (v.k[j] < K - 1 ? (R)1 : (R)0) * (mb * ((R)0.5 * (th_i[j] + thd[j])));
                    vd = bot - top;
                }
                const R dTh = -hdiv[j] - vd;
                Th_new[j] = Thn.v[j] + a.dts * (double)dTh;
                ps_new[j] = psn_[j] + a.dts * dps_[j];
            }
        }
    }
    if constexpr (MODEL == MODEL_SW) {
        return;
    } else {
        // all reads of ps_n / Th_n happen before this barrier (stage 3 writes in place)
        __syncthreads();
        if constexpr (MODEL == MODEL_HDC) {
            // FP64 column diagnostics (Eqs. 8-9); the variant VAR_PGF32 computes
            // them in FP32, as the single-precision model would
            constexpr bool P32 = VAR == VAR_PGF32;
            using RP = typename std::conditional<P32, float, double>::type;
            double *sA = lds;                       // [cpb][KM]
            RP al[L];
            const double phs = cl.valid ? a.phis[i] : 0.0;   // surface geopotential (terrain)
            if (cl.valid) {
                Pack<double, L> tho;
                Pack<float, L> th32;
#pragma unroll
                for (int j = 0; j < L; j++) {
                    const int k = v.k[j];
                    tho.v[j] = Th_new[j];
                    if constexpr (sizeof(R) == 8) {
                        sgt[j] = a.sig[k];
                        sgb[j] = a.sig[k + 1];
                    }
                    const double dpn = dsg[j] * (ps_new[j] - a.ptop);
                    const double th = Th_new[j] / dpn;
                    if constexpr (P32) {
                        const float pt = (float)a.ptop, psf = (float)ps_new[j];
                        const float pit = pt + (float)sgt[j] * (psf - pt), pib = pt + (float)sgb[j] * (psf - pt);
                        const float dpf = (float)dsg[j] * (psf - pt);
                        const float pk = 0.5f * (pit + pib);
                        const float T = ((float)Th_new[j] / dpf) * expf((float)a.kappa * logf(pk * (float)a.inv_p0));
                        al[j] = (float)a.rd * T / pk;
                        sA[lc * KM + km0 + j] = (double)(al[j] * dpf);
                    } else {
                        const double pit = a.ptop + sgt[j] * (ps_new[j] - a.ptop);
                        const double pib = a.ptop + sgb[j] * (ps_new[j] - a.ptop);
                        const double pk = 0.5 * (pit + pib);
                        const double T = th * powpos(pk * a.inv_p0, a.kappa);
                        al[j] = a.rd * T / pk;
                        sA[lc * KM + km0 + j] = al[j] * dpn;
                    }
                    th32.v[j] = (float)th;
                }
                if (a.store64) stp<double, L>(a.Th_o + (long)i * KM + km0, tho);
                if (a.th32_o) stp<float, L>(a.th32_o + (long)i * KM + km0, th32);
#pragma unroll
                for (int j = 0; j < L; j++)
                    if (v.k[j] == 0) a.ps_o[(long)i * M + v.mm0 + (M1 ? 0 : j)] = ps_new[j];
            }
            __syncthreads();
            // hydrostatic geopotential from the surface upwards (Eq. 8).  One
            // member: a lane's L values are consecutive levels and the deepest
            // one's sequential sum is extended upwards.  Several members: suffix
            // sums over k of alpha dpi by a parallel scan in LDS (Hillis-Steele,
            // double buffered; in the precision RP of the diagnostics), the same
            // sums whatever the launch shape (measured faster for the ensemble,
            // slower for one member at G6).
            if constexpr (M1) {
                if (cl.valid) {
                    Pack<double, L> alp, php;
                    RP acc = lds_sum_down<RP>(sA + lc * KM, 1, K - 1, v.k[L - 1], (RP)phs);
#pragma unroll
                    for (int j = L - 1; j >= 0; j--) {
                        const RP phit = acc + (RP)sA[lc * KM + v.k[j]];
                        alp.v[j] = (double)al[j];
                        php.v[j] = (double)((RP)0.5 * (phit + acc));
                        acc = phit;
                    }
                    stp<double, L>(a.alpha + (long)i * KM + km0, alp);
                    stp<double, L>(a.phim + (long)i * KM + km0, php);
                }
            } else {
                const double *usum;
                {
                    double *src = sA, *dst = sA + a.cpb * KM;
                    for (int d = 1; d < K; d *= 2) {
                        if (cl.valid) {
#pragma unroll
                            for (int j = 0; j < L; j++) {
                                const int o = lc * KM + v.k[j] * M + v.mm0 + (M1 ? 0 : j);
                                const bool in = v.k[j] + d < K;
                                const double hi = src[o + (in ? d * M : 0)];   // clamped: unused at the bottom
                                dst[o] = in ? (double)((RP)src[o] + (RP)hi) : src[o];
                            }
                        }
                        __syncthreads();
                        double *tmp = src;
                        src = dst;
                        dst = tmp;
                    }
                    usum = src;
                }
                if (cl.valid) {
                    Pack<double, L> alp, php;
#pragma unroll
                    for (int j = 0; j < L; j++) {
                        const int o = lc * KM + v.k[j] * M + v.mm0 + (M1 ? 0 : j);
                        const bool top = v.k[j] < K - 1;
                        const RP below = (RP)usum[o + (top ? M : 0)];   // clamped: unused in the lowest layer
                        const RP phit = (RP)phs + (RP)usum[o];           // top of the layer
                        const RP phib = top ? (RP)phs + below : (RP)phs;  // bottom of the layer
                        alp.v[j] = (double)al[j];
                        php.v[j] = (double)((RP)0.5 * (phit + phib));
                    }
                    stp<double, L>(a.alpha + (long)i * KM + km0, alp);
                    stp<double, L>(a.phim + (long)i * KM + km0, php);
                }
            }
        } else {
            // ---- implicit vertical acoustic solve of the column (FP64) ----
            // The variant VAR_PGF32 (and so SGL) computes the equation of
            // state, the column system and its solution, the specific volume,
            // the geopotential and mu in FP32 (RS); every value is still kept in
            // the FP64 arrays, rounded from its FP32 result.
            constexpr bool P32 = VAR == VAR_PGF32;
            using RS = typename std::conditional<P32, float, double>::type;
            const int K1 = K + 1;
            const long K1M = (long)K1 * M;
            const long cb = (long)i * K1M;
            double *sP = lds;                         // p*   [cpb][KM]
            double *sC = sP + a.cpb * KM;             // C    [cpb][KM]
            double *sSub = sC + a.cpb * KM;           // rows [cpb][KM]
            double *sDia = sSub + a.cpb * KM;
            double *sSup = sDia + a.cpb * KM;
            double *sRhs = sSup + a.cpb * KM;
            double *sCp = sRhs + a.cpb * KM;
            double *sDp = sCp + a.cpb * KM;
            double *sPhi = sDp + a.cpb * KM;          // [cpb][(K+1) M]
            double *sPn = sPhi + a.cpb * K1 * M;      // [cpb][KM] updated pressure
            const int base = lc * KM;
            double dpn[L], phs_k[L], phs_k1[L], ws_k[L];
            if (cl.valid) {
                Pack<double, L> tho;
                Pack<float, L> th32;
                ld_iface<L, M1>(a.phistar, cb, v, M, 0, phs_k);
                ld_iface<L, M1>(a.phistar, cb, v, M, 1, phs_k1);
                ld_iface<L, M1>(a.wstar, cb, v, M, 0, ws_k);
#pragma unroll
                for (int j = 0; j < L; j++) {
                    tho.v[j] = Th_new[j];
                    dpn[j] = dsg[j] * (ps_new[j] - a.ptop);
                    th32.v[j] = (float)(Th_new[j] / dpn[j]);
                    const RS dphi = (RS)phs_k[j] - (RS)phs_k1[j];
                    const RS p = (RS)a.p0 * powpos((RS)a.rd * (RS)Th_new[j] / ((RS)a.p0 * dphi), (RS)a.gamma);
                    sP[base + km0 + j] = (double)p;
                    sC[base + km0 + j] = (double)((RS)a.gamma * (RS)a.grav * (RS)a.dts * p / dphi);
                }
                if (a.store64) stp<double, L>(a.Th_o + (long)i * KM + km0, tho);
                if (a.th32_o) stp<float, L>(a.th32_o + (long)i * KM + km0, th32);
#pragma unroll
                for (int j = 0; j < L; j++)
                    if (v.k[j] == 0) a.ps_o[(long)i * M + v.mm0 + (M1 ? 0 : j)] = ps_new[j];
            }
            __syncthreads();
            if (cl.valid) {
#pragma unroll
                for (int j = 0; j < L; j++) {
                    const int k = v.k[j], mm = v.mm0 + (M1 ? 0 : j);
                    if (k < 1) continue;
                    // row r = k-1 for interior interface k (between layers k-1 and k)
                    const double dpm = a.dsig[k - 1] * (ps_new[j] - a.ptop);
                    const RS D = (RS)a.grav * (RS)a.dts / ((RS)0.5 * ((RS)dpm + (RS)dpn[j]));
                    const RS Cm = (RS)sC[base + (k - 1) * M + mm], Ck = (RS)sC[base + k * M + mm];
                    const int r = (k - 1) * M + mm;
                    sSub[base + r] = (double)(-D * Cm);
                    sDia[base + r] = (double)((RS)1 + D * (Cm + Ck));
                    sSup[base + r] = (double)(-D * Ck);
                    sRhs[base + r] = (double)((RS)ws_k[j] + D * ((RS)sP[base + k * M + mm] - (RS)sP[base + (k - 1) * M + mm]) -
                                              (RS)a.grav * (RS)a.dts);
                }
            }
            __syncthreads();
            // Parallel cyclic reduction over the n = K-1 interior interfaces of
            // each member: the step with stride st eliminates, in every row at
            // once, the couplings to the rows st above and below (rows beyond
            // the ends count as absent); after the strides 1, 2, 4, ... < n the
            // rows are decoupled and x_r = rhs_r / dia_r.  The rows of a lane are
            // its own interfaces, so the arithmetic of a row does not depend on
            // the launch shape.  p* and C are dead here and hold the second
            // buffer with sCp and sDp.
            const int n = K - 1;
            double *cur[4] = {sSub, sDia, sSup, sRhs}, *nxt[4] = {sP, sC, sCp, sDp};
            for (int st = 1; st < n; st *= 2) {
                if (cl.valid) {
#pragma unroll
                    for (int j = 0; j < L; j++) {
                        const int k = v.k[j], mm = v.mm0 + (M1 ? 0 : j);
                        if (k < 1) continue;
                        const int r = k - 1, o = base + r * M + mm;
                        RS bb = (RS)cur[1][o], dd = (RS)cur[3][o], na = 0, nc = 0;
                        if (r - st >= 0) {
                            const int q = o - st * M;
                            const RS f = (RS)cur[0][o] / (RS)cur[1][q];
                            bb = fmar(-(RS)cur[2][q], f, bb);
                            dd = fmar(-(RS)cur[3][q], f, dd);
                            na = -(RS)cur[0][q] * f;
                        }
                        if (r + st < n) {
                            const int q = o + st * M;
                            const RS f = (RS)cur[2][o] / (RS)cur[1][q];
                            bb = fmar(-(RS)cur[0][q], f, bb);
                            dd = fmar(-(RS)cur[3][q], f, dd);
                            nc = -(RS)cur[2][q] * f;
                        }
                        nxt[0][o] = (double)na;
                        nxt[1][o] = (double)bb;
                        nxt[2][o] = (double)nc;
                        nxt[3][o] = (double)dd;
                    }
                }
                __syncthreads();
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    double *t = cur[q];
                    cur[q] = nxt[q];
                    nxt[q] = t;
                }
            }
            double phk[L];
            if (cl.valid) {
                double wk[L];
#pragma unroll
                for (int j = 0; j < L; j++) {
                    const int k = v.k[j], mm = v.mm0 + (M1 ? 0 : j);
                    const RS wr = (k == 0) ? (RS)0 : (RS)cur[3][base + (k - 1) * M + mm] / (RS)cur[1][base + (k - 1) * M + mm];
                    wk[j] = (double)wr;
                    phk[j] = (double)((RS)phs_k[j] + (RS)a.grav * (RS)a.dts * wr);
                    sPhi[lc * K1 * M + k * M + mm] = phk[j];
                    if (k == K - 1) sPhi[lc * K1 * M + K * M + mm] = phs_k1[j];   // surface: phi_s
                }
                st_iface<L, M1>(a.w_o, cb, v, M, 0, wk);
                st_iface<L, M1>(a.phi_o, cb, v, M, 0, phk);
#pragma unroll
                for (int j = 0; j < L; j++) {
                    if (v.k[j] == K - 1) {
                        const int mm = v.mm0 + (M1 ? 0 : j);
                        a.w_o[cb + (long)K * M + mm] = a.wstar[cb + (long)K * M + mm];   // kinematic
                        a.phi_o[cb + (long)K * M + mm] = phs_k1[j];
                    }
                }
            }
            __syncthreads();
            if (cl.valid) {
                Pack<double, L> alp, pmp, php;
#pragma unroll
                for (int j = 0; j < L; j++) {
                    const int k = v.k[j], mm = v.mm0 + (M1 ? 0 : j);
                    const double phb = sPhi[lc * K1 * M + (k + 1) * M + mm];
                    const RS dphi = (RS)phk[j] - (RS)phb;
                    const RS pk = (RS)a.p0 * powpos((RS)a.rd * (RS)Th_new[j] / ((RS)a.p0 * dphi), (RS)a.gamma);
                    sPn[base + k * M + mm] = (double)pk;
                    alp.v[j] = (double)(dphi / (RS)dpn[j]);
                    pmp.v[j] = (double)pk;
                    php.v[j] = (double)((RS)0.5 * ((RS)phk[j] + (RS)phb));
                }
                stp<double, L>(a.alpha + (long)i * KM + km0, alp);
                stp<double, L>(a.pm + (long)i * KM + km0, pmp);
                stp<double, L>(a.phim + (long)i * KM + km0, php);
            }
            __syncthreads();
            if (cl.valid) {
                // mu = dp/dpi at interfaces, copied to the ends, averaged to the layer
                Pack<double, L> mup;
#pragma unroll
                for (int j = 0; j < L; j++) {
                    const int mm = v.mm0 + (M1 ? 0 : j);
                    const double psj = ps_new[j];
                    auto mu_at = [&](int kk) -> RS {
                        if (K == 1) return (RS)1;
                        if (kk < 1) kk = 1;
                        if (kk > K - 1) kk = K - 1;
                        const double dp_a = a.dsig[kk - 1] * (psj - a.ptop);
                        const double dp_b = a.dsig[kk] * (psj - a.ptop);
                        return ((RS)sPn[base + kk * M + mm] - (RS)sPn[base + (kk - 1) * M + mm]) /
                               ((RS)0.5 * ((RS)dp_a + (RS)dp_b));
                    };
                    mup.v[j] = (double)((RS)0.5 * (mu_at(v.k[j]) + mu_at(v.k[j] + 1)));
                }
                stp<double, L>(a.mum + (long)i * KM + km0, mup);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// edge: momentum
// ---------------------------------------------------------------------------
// LDS of the edge kernel: per edge of the work-group its two cells and
// 1/d_e, then the two cells' surface pressures of the stage input and of
// the pressure-gradient term [4][M]; then sigma [K+1] and dsigma [K].
// Shapes whose edges would not fit 64 KiB read them directly instead.
__host__ __device__ inline size_t edge_lds_bytes(int flat_block, int lanes, int K, int M) {
    return ((size_t)vertex_stage_max(flat_block, lanes) * (3 + 4 * (size_t)M) + 2 * (size_t)K + 1) * 8;
}

template <int MODEL, typename R, int L, bool M1, int VAR, bool STAGED>
__global__ void __launch_bounds__(1024) k_edge(StageArgs a) {
    // boxed variant: -grad K and the vertical advection of u in FP64 (from the
    // FP64 kinetic energy and velocity), rounded to FP32 once with the
    // pressure-gradient term as one tendency
    constexpr bool BOX = VAR == VAR_BOX;
    using RU = typename std::conditional<BOX, double, R>::type;
    extern __shared__ double elds[];
    const DevMesh &m = a.mesh;
    const int K = a.K, M = M1 ? 1 : a.M, KM = K * M;
    const int lanes = KM / L;
    const long b0 = (long)xcd_block() * a.flat_block;   // flat_block = threads per work-group
    const long nall = (long)m.E * lanes;
    const long idx = b0 + threadIdx.x;
    const bool valid = idx < nall;
    const int e = (int)((valid ? idx : nall - 1) / lanes);
    const int km0 = (int)((valid ? idx : nall - 1) - (long)e * lanes) * L;
    const long base = (long)e * KM + km0;
    const Vals<L, M1> v(km0, M);

    // Coriolis - grad K: the two cells' shares (issued before the staging)
    R adv[L];
    {
        const R *qh = a.qh_in<R>();
        const Pack<R, L> q1 = ldp<R, L>(qh + (long)e * 2 * KM + km0), q2 = ldp<R, L>(qh + ((long)e * 2 + 1) * KM + km0);
#pragma unroll
        for (int j = 0; j < L; j++) adv[j] = q1.v[j] + q2.v[j];
    }
    // The work-group's edges share their cells, 1/d_e, the cells' surface
    // pressures and the level fractions among all K M / L lanes of each edge:
    // staged once in LDS, so the lanes gather only the fields of the levels.
    const int e0 = (int)(b0 / lanes);
    const int nem = vertex_stage_max(a.flat_block, lanes);
    const int row_len = 3 + 4 * M;
    double *sR = elds;                              // [nem][3 + 4 M]
    double *sS = sR + (long)nem * row_len;          // sigma [K+1]
    double *sD = sS + K + 1;                        // dsigma [K]
    if constexpr (STAGED) {
        const long lastl = (b0 + a.flat_block < nall ? b0 + a.flat_block : nall) - 1;
        const int ne = (int)(lastl / lanes) - e0 + 1;
        const int nps = ne * 4 * M;
        for (int x = threadIdx.x; x < ne + nps + 2 * K + 1; x += blockDim.x) {
            if (x < ne) {
                const long ex = e0 + x;
                const Pack<int, 2> cc = ldp<int, 2>(m.e_cell + 2 * ex);
                double *r = sR + (long)x * row_len;
                r[0] = (double)cc.v[0];
                r[1] = (double)cc.v[1];
                r[2] = m.e_dinv[ex];
            } else if (x < ne + nps) {
                const int y = x - ne, es = y / (4 * M), q = (y - es * 4 * M) / M, mm = y - es * 4 * M - q * M;
                const int c = m.e_cell[2 * (long)(e0 + es) + (q & 1)];
                sR[(long)es * row_len + 3 + q * M + mm] = (q < 2 ? a.ps_s : a.ps_pg)[(long)c * M + mm];
            } else if (x < ne + nps + K + 1) {
                sS[x - ne - nps] = a.sig[x - ne - nps];
            } else {
                sD[x - ne - nps - K - 1] = a.dsig[x - ne - nps - K - 1];
            }
        }
        __syncthreads();
    }
    if (!valid) return;
    const double *row = sR + (long)(e - e0) * row_len;
    int c1, c2;
    double dinv_e;
    if constexpr (STAGED) {
        c1 = (int)row[0];
        c2 = (int)row[1];
        dinv_e = row[2];
    } else {
        const Pack<int, 2> cc = ldp<int, 2>(m.e_cell + 2 * (long)e);
        c1 = cc.v[0];
        c2 = cc.v[1];
        dinv_e = m.e_dinv[e];
    }
    // surface pressure q (0, 1: the stage input at c1, c2; 2, 3: the
    // pressure-gradient term's at c1, c2) and the level fractions
    auto cell_ps = [&](int q, double out[L]) {
        if constexpr (STAGED) ld2d_s<L, M1>(row + 3 + q * M, v.mm0, out);
        else ld2d<L, M1>(q < 2 ? a.ps_s : a.ps_pg, (q & 1) ? c2 : c1, M, v.mm0, out);
    };
    auto sig_at = [&](int k) { return STAGED ? sS[k] : a.sig[k]; };
    auto dsig_at = [&](int k) { return STAGED ? sD[k] : a.dsig[k]; };

    double box[L];
    if constexpr (BOX) {
        const double *ke = (const double *)a.ke;
        const Pack<double, L> k1 = ldp<double, L>(ke + (long)c1 * KM + km0), k2 = ldp<double, L>(ke + (long)c2 * KM + km0);
#pragma unroll
        for (int j = 0; j < L; j++) box[j] = -(k2.v[j] - k1.v[j]) * dinv_e;
    }

    if constexpr (MODEL != MODEL_SW) {
        // centred vertical advection of u by the interface mass flux
        const RU *us;
        if constexpr (BOX) us = a.u_s;
        else us = u_prev_ptr<R>(a);
        const long K1M = (long)(K + 1) * M;
        double p1[L], p2[L], dsg[L];
        cell_ps(0, p1);
        cell_ps(1, p2);
#pragma unroll
        for (int j = 0; j < L; j++) dsg[j] = dsig_at(v.k[j]);
        const Pack<RU, L> uk = ldp<RU, L>(us + base);
        RU uup[L], udn[L];
        // the interface mass flux: its FP32 copy in the FP32 policies
        using MT = typename std::conditional<mdot32_used<R, VAR>(), float, double>::type;
        const MT *mdp;
        if constexpr (sizeof(MT) == 4) mdp = a.mdot32;
        else mdp = a.mdot;
        MT mt[L], mb[L];
        // the levels above and below are read from clamped indices (no load
        // under a condition); the values past the lid and the surface are unused
        if constexpr (M1) {
            const RU ua = us[base + (v.k0 > 0 ? -1 : 0)];
            const RU ub = us[base + (v.k[L - 1] < K - 1 ? L : L - 1)];
#pragma unroll
            for (int j = 0; j < L; j++) {
                uup[j] = (j > 0) ? uk.v[j - 1] : ua;   // ua, ub: unused at the lid and the surface
                udn[j] = (j < L - 1) ? uk.v[j + 1] : ub;
            }
            const MT *m1p = mdp + (long)c1 * K1M + v.k0, *m2p = mdp + (long)c2 * K1M + v.k0;
            MT i1[L + 1], i2[L + 1];
#pragma unroll
            for (int j = 0; j <= L; j++) {
                i1[j] = m1p[j];
                i2[j] = m2p[j];
            }
#pragma unroll
            for (int j = 0; j < L; j++) {
                mt[j] = (MT)0.5 * (i1[j] + i2[j]);
                mb[j] = (MT)0.5 * (i1[j + 1] + i2[j + 1]);
            }
        } else if constexpr (sizeof(RU) == 4 && sizeof(MT) == 4) {
            // Several members: the lane M / L further in the wave holds the same
            // members one level down (of the same edge, or past the surface,
            // where the value is unused), so the level above and below of u and
            // the lower interface's flux come across the wave, not from memory;
            // only the lanes whose partner is in the next or previous wave load.
            const Pack<MT, L> t1 = ldp<MT, L>(mdp + (long)c1 * K1M + (long)v.k0 * M + v.mm0);
            const Pack<MT, L> t2 = ldp<MT, L>(mdp + (long)c2 * K1M + (long)v.k0 * M + v.mm0);
#pragma unroll
            for (int j = 0; j < L; j++) mt[j] = (MT)0.5 * (t1.v[j] + t2.v[j]);
            const int wl = (int)(threadIdx.x & 63), dl = M / L;
#pragma unroll
            for (int j = 0; j < L; j++) {
                uup[j] = __shfl_up(uk.v[j], dl, 64);
                udn[j] = __shfl_down(uk.v[j], dl, 64);
                mb[j] = __shfl_down(mt[j], dl, 64);
                // past the lid and the surface the partner may be another edge or
                // an idle lane: the values the loads would give there (unused, but
                // finite, as they are multiplied by zero)
                if (v.k0 == 0) uup[j] = uk.v[j];
                if (v.k0 == K - 1) {
                    udn[j] = uk.v[j];
                    mb[j] = (MT)0;
                }
            }
            if (wl < dl) {
                const Pack<RU, L> pu = ldp<RU, L>(us + base - (v.k0 > 0 ? M : 0));
#pragma unroll
                for (int j = 0; j < L; j++) uup[j] = pu.v[j];
            }
            if (wl + dl > 63) {
                const Pack<RU, L> pd = ldp<RU, L>(us + base + (v.k0 < K - 1 ? M : 0));
                const Pack<MT, L> b1 = ldp<MT, L>(mdp + (long)c1 * K1M + (long)(v.k0 + 1) * M + v.mm0);
                const Pack<MT, L> b2 = ldp<MT, L>(mdp + (long)c2 * K1M + (long)(v.k0 + 1) * M + v.mm0);
#pragma unroll
                for (int j = 0; j < L; j++) {
                    udn[j] = pd.v[j];
                    mb[j] = (MT)0.5 * (b1.v[j] + b2.v[j]);
                }
            }
        } else {
            const Pack<RU, L> pu = ldp<RU, L>(us + base - (v.k0 > 0 ? M : 0));
            const Pack<RU, L> pd = ldp<RU, L>(us + base + (v.k0 < K - 1 ? M : 0));
            const Pack<MT, L> t1 = ldp<MT, L>(mdp + (long)c1 * K1M + (long)v.k0 * M + v.mm0);
            const Pack<MT, L> t2 = ldp<MT, L>(mdp + (long)c2 * K1M + (long)v.k0 * M + v.mm0);
            const Pack<MT, L> b1 = ldp<MT, L>(mdp + (long)c1 * K1M + (long)(v.k0 + 1) * M + v.mm0);
            const Pack<MT, L> b2 = ldp<MT, L>(mdp + (long)c2 * K1M + (long)(v.k0 + 1) * M + v.mm0);
#pragma unroll
            for (int j = 0; j < L; j++) {
                uup[j] = pu.v[j];
                udn[j] = pd.v[j];
                mt[j] = (MT)0.5 * (t1.v[j] + t2.v[j]);
                mb[j] = (MT)0.5 * (b1.v[j] + b2.v[j]);
            }
        }
#pragma unroll
        for (int j = 0; j < L; j++) {
            const double dpe = 0.5 * (lmass<MODEL>(dsg[j], p1[j], a.ptop) + lmass<MODEL>(dsg[j], p2[j], a.ptop));
            // the terms through the lid and the surface are multiplied by zero
            // rather than skipped (a branch would hold the loads behind it)
            const RU fb = v.k[j] < K - 1 ? (RU)1 : (RU)0, ft = v.k[j] > 0 ? (RU)1 : (RU)0;
            RU va = 0;
            va += fb * ((RU)mb[j] * (udn[j] - uk.v[j]));
            va += ft * ((RU)mt[j] * (uk.v[j] - uup[j]));
            va = va / (RU)(2.0 * dpe);
            if constexpr (BOX) box[j] -= va;
            else adv[j] = adv[j] - va;
        }
    }

    // pressure-gradient force and gravity in FP64 from the updated mass/Theta
    // (forward-backward; ps_pg is the stage's input mass when that is off)
    const double dinv64 = dinv_e;
    double pgf[L];
    if constexpr (MODEL == MODEL_SW) {
        double h1[L], h2[L];
        cell_ps(2, h1);
        cell_ps(3, h2);
        const double b1 = a.b[c1], b2 = a.b[c2];
#pragma unroll
        for (int j = 0; j < L; j++) pgf[j] = -a.grav * ((h2[j] + b2) - (h1[j] + b1)) * dinv64;
    } else {
        const long x1 = (long)c1 * KM + km0, x2 = (long)c2 * KM + km0;
        const Pack<double, L> al1 = ldp<double, L>(a.alpha + x1), al2 = ldp<double, L>(a.alpha + x2);
        const Pack<double, L> ph1 = ldp<double, L>(a.phim + x1), ph2 = ldp<double, L>(a.phim + x2);
        if constexpr (MODEL == MODEL_HDC) {
            double s1[L], s2[L];
            cell_ps(2, s1);
            cell_ps(3, s2);
#pragma unroll
            for (int j = 0; j < L; j++) {
                const int k = v.k[j];
                const double sgk = sig_at(k), sgk1 = sig_at(k + 1);
                if constexpr (VAR == VAR_PGF32) {
                    // the single-precision pressure-gradient term of the FP32 variant
                    const float pt = (float)a.ptop, st_ = (float)sgk, sb = (float)sgk1;
                    const float f1 = (float)s1[j], f2 = (float)s2[j];
                    const float q1 = 0.5f * ((pt + st_ * (f1 - pt)) + (pt + sb * (f1 - pt)));
                    const float q2 = 0.5f * ((pt + st_ * (f2 - pt)) + (pt + sb * (f2 - pt)));
                    const float ae = 0.5f * ((float)al1.v[j] + (float)al2.v[j]);
                    pgf[j] = (double)(-(ae * (q2 - q1) + ((float)ph2.v[j] - (float)ph1.v[j])) * (float)dinv64);
                    continue;
                }
                const double q1 = 0.5 * ((a.ptop + sgk * (s1[j] - a.ptop)) + (a.ptop + sgk1 * (s1[j] - a.ptop)));
                const double q2 = 0.5 * ((a.ptop + sgk * (s2[j] - a.ptop)) + (a.ptop + sgk1 * (s2[j] - a.ptop)));
                const double ae = 0.5 * (al1.v[j] + al2.v[j]);
                pgf[j] = -(ae * (q2 - q1) + (ph2.v[j] - ph1.v[j])) * dinv64;
            }
        } else {
            const Pack<double, L> q1 = ldp<double, L>(a.pm + x1), q2 = ldp<double, L>(a.pm + x2);
            const Pack<double, L> u1 = ldp<double, L>(a.mum + x1), u2 = ldp<double, L>(a.mum + x2);
#pragma unroll
            for (int j = 0; j < L; j++) {
                if constexpr (VAR == VAR_PGF32) {
                    // the single-precision pressure-gradient term of the FP32 variant
                    const float ae = 0.5f * ((float)al1.v[j] + (float)al2.v[j]);
                    const float me = 0.5f * ((float)u1.v[j] + (float)u2.v[j]);
                    pgf[j] = (double)(-(ae * ((float)q2.v[j] - (float)q1.v[j]) + me * ((float)ph2.v[j] - (float)ph1.v[j])) *
                                      (float)dinv64);
                    continue;
                }
                const double ae = 0.5 * (al1.v[j] + al2.v[j]);
                const double me = 0.5 * (u1.v[j] + u2.v[j]);
                pgf[j] = -(ae * (q2.v[j] - q1.v[j]) + me * (ph2.v[j] - ph1.v[j])) * dinv64;
            }
        }
    }
    const Pack<double, L> un = ldp<double, L>(a.u_n + base);
    Pack<double, L> uo;
    Pack<float, L> u32;
#pragma unroll
    for (int j = 0; j < L; j++) {
        if constexpr (BOX) uo.v[j] = un.v[j] + a.dts * (double)(adv[j] + (float)(box[j] + pgf[j]));
        else uo.v[j] = un.v[j] + a.dts * ((double)adv[j] + pgf[j]);
        u32.v[j] = (float)uo.v[j];
    }
    if (a.store64) stp<double, L>(a.u_o + base, uo);
    if (a.u32_o) stp<float, L>(a.u32_o + base, u32);
}

// ---------------------------------------------------------------------------
// shadows: FP32 copies of u and theta for the mixed policy
// ---------------------------------------------------------------------------
template <int MODEL>
__global__ void k_shadows(StageArgs a) {
    const int KM = a.K * a.M;
    const long idx = (long)xcd_block() * a.flat_block + threadIdx.x;   // flat_block = threads per work-group
    const long nE = (long)a.mesh.E * KM, nC = (long)a.mesh.N * KM;
    if (idx < nE) a.u32_o[idx] = (float)a.u_o[idx];
    if (MODEL != MODEL_SW && a.th32_o && idx < nC) {
        const int i = (int)(idx / KM);
        const int km = (int)(idx - (long)i * KM);
        const int k = km / a.M, mm = km - k * a.M;
        a.th32_o[idx] = (float)(a.Th_o[idx] / lmass<MODEL>(a.dsig[k], a.ps_o[(long)i * a.M + mm], a.ptop));
    }
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
namespace {
inline unsigned nblocks(long n, int b) { return (unsigned)((n + b - 1) / b); }

// the vertex kernel, its tables staged in LDS where the work-group's vertices fit
template <int MODEL, typename R, int L, bool M1, int VV> void launch_vertex(const StageArgs &a, hipStream_t s) {
    const int lanes = a.K * a.M / L, fb = a.flat_block;
    const size_t lds = vertex_lds_bytes(fb, lanes, a.K, a.M);
    if (lds <= kVertexLdsMax)
        hipLaunchKernelGGL((k_vertex<MODEL, R, L, M1, VV, true>), dim3(nblocks((long)a.mesh.V * lanes, fb)), dim3(fb),
                           lds, s, a);
    else
        hipLaunchKernelGGL((k_vertex<MODEL, R, L, M1, VV, false>), dim3(nblocks((long)a.mesh.V * lanes, fb)),
                           dim3(fb), 0, s, a);
}

// the edge kernel, its per-edge values staged in LDS where the work-group's edges fit
template <int MODEL, typename R, int L, bool M1, int VB> void launch_edge(const StageArgs &a, hipStream_t s) {
    const int lanes = a.K * a.M / L, fb = a.flat_block;
    const size_t lds = edge_lds_bytes(fb, lanes, a.K, a.M);
    if (lds <= kVertexLdsMax)
        hipLaunchKernelGGL((k_edge<MODEL, R, L, M1, VB, true>), dim3(nblocks((long)a.mesh.E * lanes, fb)), dim3(fb),
                           lds, s, a);
    else
        hipLaunchKernelGGL((k_edge<MODEL, R, L, M1, VB, false>), dim3(nblocks((long)a.mesh.E * lanes, fb)), dim3(fb),
                           0, s, a);
}

// VAR selects the mixed-policy variant of the FP32 instances; a kernel the
// variant does not change runs its default instance
template <int MODEL, typename R, int L, bool M1, int VAR>
hipError_t launch_stage_t(const StageArgs &a, int which, hipStream_t s) {
    // the all-FP32 variant: FP32 divergence in cell_a, its own vertex kernel, the
    // FP32 pressure-gradient instances of cell_b and edge
    constexpr int VA = VAR == VAR_PGF32 ? VAR_MIX : VAR == VAR_SGL ? VAR_F32_DIV : VAR;   // cell_a
    constexpr int VB = (VAR == VAR_BOX || VAR == VAR_PGF32) ? VAR : VAR == VAR_SGL ? VAR_PGF32 : VAR_MIX;
    constexpr int VV = VAR == VAR_SGL ? VAR_SGL : VAR_MIX;                                // vertex
    const int KM = a.K * a.M;
    const int lanes = KM / L;
    const int colthreads = a.cpb * lanes;
    const unsigned colblocks = nblocks(a.mesh.N, a.cpb);
    const int fb = a.flat_block;
    const int pol = sizeof(R) == 8 ? POLICY_DBL : POLICY_MIX;
    const size_t lds_a = stage_lds_bytes(MODEL, pol, KERNEL_CELL_A, a.cpb, a.K, a.M);
    const size_t lds_b = stage_lds_bytes(MODEL, pol, KERNEL_CELL_B, a.cpb, a.K, a.M);
    // One cell per work-group of an ensemble takes the uniform-cell instance of
    // the column kernels (one member: measured slower at G8 x 60 and G9 x 30,
    // whose columns of 30 to 60 lanes leave most of a wave idle or need no
    // fewer registers than the autotuned general shapes).
    constexpr bool UB = !M1;
    switch (which) {
    case KERNEL_CELL_A:
        if (UB && a.cpb == 1)
            hipLaunchKernelGGL((k_cell_a<MODEL, R, L, M1, VA, UB>), dim3(colblocks), dim3(colthreads), lds_a, s, a);
        else
            hipLaunchKernelGGL((k_cell_a<MODEL, R, L, M1, VA, false>), dim3(colblocks), dim3(colthreads), lds_a, s, a);
        break;
    case KERNEL_VERTEX:
        launch_vertex<MODEL, R, L, M1, VV>(a, s);
        break;
    case KERNEL_CELL_B:
        if (UB && a.cpb == 1)
            hipLaunchKernelGGL((k_cell_b<MODEL, R, L, M1, VB, UB>), dim3(colblocks), dim3(colthreads), lds_b, s, a);
        else
            hipLaunchKernelGGL((k_cell_b<MODEL, R, L, M1, VB, false>), dim3(colblocks), dim3(colthreads), lds_b, s, a);
        break;
    case KERNEL_EDGE:
        launch_edge<MODEL, R, L, M1, VB>(a, s);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Four values per lane: the flat kernels (vertex, edge), and for an ensemble
// (four members per lane, one cell per work-group) the uniform-cell column
// kernels of the FP32 policies
template <int MODEL, typename R, bool M1, int VAR>
hipError_t launch_flat4(const StageArgs &a, int which, hipStream_t s) {
    constexpr int VA = VAR == VAR_PGF32 ? VAR_MIX : VAR == VAR_SGL ? VAR_F32_DIV : VAR;
    constexpr int VB = (VAR == VAR_BOX || VAR == VAR_PGF32) ? VAR : VAR == VAR_SGL ? VAR_PGF32 : VAR_MIX;
    constexpr int VV = VAR == VAR_SGL ? VAR_SGL : VAR_MIX;
    constexpr bool C4 = !M1 && sizeof(R) == 4;
    if (which == KERNEL_VERTEX) {
        launch_vertex<MODEL, R, 4, M1, VV>(a, s);
    } else if (which == KERNEL_EDGE) {
        launch_edge<MODEL, R, 4, M1, VB>(a, s);
    } else if (C4 && a.cpb == 1 && (which == KERNEL_CELL_A || which == KERNEL_CELL_B)) {
        if constexpr (C4) {
            const int pol = POLICY_MIX;
            const unsigned nb = a.mesh.N;
            const int threads = a.K * a.M / 4;
            if (which == KERNEL_CELL_A)
                hipLaunchKernelGGL((k_cell_a<MODEL, R, 4, false, VA, true>), dim3(nb), dim3(threads),
                                   stage_lds_bytes(MODEL, pol, KERNEL_CELL_A, 1, a.K, a.M), s, a);
            else
                hipLaunchKernelGGL((k_cell_b<MODEL, R, 4, false, VB, true>), dim3(nb), dim3(threads),
                                   stage_lds_bytes(MODEL, pol, KERNEL_CELL_B, 1, a.K, a.M), s, a);
        }
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int MODEL, typename R, int VAR>
hipError_t launch_stage_r(const StageArgs &a, int which, hipStream_t s) {
    const int L = a.vpl;
    if (a.M == 1) {
        if (L == 4) return launch_flat4<MODEL, R, true, VAR>(a, which, s);
        return L == 2 ? launch_stage_t<MODEL, R, 2, true, VAR>(a, which, s)
                      : launch_stage_t<MODEL, R, 1, true, VAR>(a, which, s);
    }
    if (L == 4) return launch_flat4<MODEL, R, false, VAR>(a, which, s);
    return L == 2 ? launch_stage_t<MODEL, R, 2, false, VAR>(a, which, s)
                  : launch_stage_t<MODEL, R, 1, false, VAR>(a, which, s);
}

// the variants exist for the layered models only
template <int VAR> hipError_t launch_variant(int model, const StageArgs &a, int which, hipStream_t s) {
    if (model == MODEL_HDC) return launch_stage_r<MODEL_HDC, float, VAR>(a, which, s);
    if (model == MODEL_NDC) return launch_stage_r<MODEL_NDC, float, VAR>(a, which, s);
    return hipErrorInvalidValue;
}
}  // namespace

int values_per_lane(int K, int M) { return (M == 1 ? (K % 2 == 0) : (M % 2 == 0)) ? 2 : 1; }

size_t stage_lds_bytes(int model, int policy, int which, int cpb, int K, int M) {
    if (which != KERNEL_CELL_A && which != KERNEL_CELL_B) return 0;
    return col_lds_bytes(model, which, cpb, K, M) +
           coltab_layout(model, which, cpb, M, policy == POLICY_DBL ? 8 : 4).bytes;
}

hipError_t launch_stage_kernel(int model, int policy, const StageArgs &a, int which, hipStream_t s) {
    switch (policy) {
    case POLICY_DBL:
        if (model == MODEL_SW) return launch_stage_r<MODEL_SW, double, VAR_MIX>(a, which, s);
        if (model == MODEL_HDC) return launch_stage_r<MODEL_HDC, double, VAR_MIX>(a, which, s);
        return launch_stage_r<MODEL_NDC, double, VAR_MIX>(a, which, s);
    case POLICY_MIX:
        if (model == MODEL_SW) return launch_stage_r<MODEL_SW, float, VAR_MIX>(a, which, s);
        return launch_variant<VAR_MIX>(model, a, which, s);
    case POLICY_MIX_BOX: return launch_variant<VAR_BOX>(model, a, which, s);
    case POLICY_MIX_DBL_MASS: return launch_variant<VAR_DBL_MASS>(model, a, which, s);
    case POLICY_MIX_F32_DIV: return launch_variant<VAR_F32_DIV>(model, a, which, s);
    case POLICY_MIX_PGF32: return launch_variant<VAR_PGF32>(model, a, which, s);
    case POLICY_SGL: return launch_variant<VAR_SGL>(model, a, which, s);
    }
    return hipErrorInvalidValue;
}

// The horizontal mass flux as the last stage's divergence used it (the same
// operations as in k_cell_a, so the values are bitwise those of the stage:
// FP32 from the FP32 velocity shadow, or FP64 from the FP64 velocity) and the
// vertical mass flux of that stage, added to FP64 accumulators.  M = 1.
template <int MODEL, bool F64>
__global__ void k_flux_acc(StageArgs a, double *Facc, double *Macc) {
    const long x = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int K = a.K;
    if (x < (long)a.mesh.E * K) {
        const int e = (int)(x / K), k = (int)(x - (long)e * K);
        const int c1 = a.mesh.e_cell[2 * e], c2 = a.mesh.e_cell[2 * e + 1];
        const double dsg = a.dsig[k];
        const double dpe = 0.5 * (lmass<MODEL>(dsg, a.ps_s[c1], a.ptop) + lmass<MODEL>(dsg, a.ps_s[c2], a.ptop));
        double f;
        if constexpr (F64) f = dpe * a.u_s[x];
        else f = (double)((float)dpe * a.u32_s[x]);
        Facc[x] += f;
    }
    if (x < (long)a.mesh.N * (K + 1)) Macc[x] += a.mdot[x];
}

hipError_t launch_flux_acc(int model, int policy, const StageArgs &a, double *Facc, double *Macc, hipStream_t s) {
    const long n = (long)(a.mesh.E > a.mesh.N + 1 ? a.mesh.E : a.mesh.N + 1) * (a.K + 1);
    const bool f64 = policy == POLICY_DBL || policy == POLICY_MIX_DBL_MASS;
    const dim3 g(nblocks(n, 256)), b(256);
    if (model == MODEL_HDC) {
        if (f64) hipLaunchKernelGGL((k_flux_acc<MODEL_HDC, true>), g, b, 0, s, a, Facc, Macc);
        else hipLaunchKernelGGL((k_flux_acc<MODEL_HDC, false>), g, b, 0, s, a, Facc, Macc);
    } else if (model == MODEL_NDC) {
        if (f64) hipLaunchKernelGGL((k_flux_acc<MODEL_NDC, true>), g, b, 0, s, a, Facc, Macc);
        else hipLaunchKernelGGL((k_flux_acc<MODEL_NDC, false>), g, b, 0, s, a, Facc, Macc);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// relative vorticity (1/A_v) sum s' d u of the FP64 velocity (Eq. 5 zeta; the
// error measure of Eqs. 1-2 uses it), one lane per vertex-level
__global__ void k_vorticity(DevMesh m, const double *u, double *out, int KM) {
    const long x = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= (long)m.V * KM) return;
    const int v = (int)(x / KM), km = (int)(x - (long)v * KM);
    double z = 0.0;
#pragma unroll
    for (int r = 0; r < 3; r++) z += m.v_curl[4 * (long)v + r] * u[(long)m.v_edge[4 * (long)v + r] * KM + km];
    out[x] = z;
}

hipError_t launch_vorticity(const DevMesh &m, const double *u, double *out, int KM, hipStream_t s) {
    const long n = (long)m.V * KM;
    hipLaunchKernelGGL(k_vorticity, dim3(nblocks(n, 256)), dim3(256), 0, s, m, u, out, KM);
    return hipGetLastError();
}

// Column energy per unit area of every (cell, member), in FP64 from the FP64
// state: (1/g) sum_k dpi_k (K_k + c_v T_k + phi_k), with the cell kinetic
// energy K = sum_j (l d / 4A) u_j^2 and phi_k the mean of the layer's two
// interface geopotentials.  Hydrostatic: T = theta (p_k/p0)^kappa at the
// mid-layer pressure, geopotential integrated upwards from phi_s (Eq. 8).
// Non-hydrostatic: p_k from Eq. 9, T = p_k (dphi_k/dpi_k) / R_d, plus the
// mean of w^2/2 at the layer's interfaces.  Shallow water: h (K + g (h/2 + b)).
// One lane per (cell, member), levels in sequence.
__global__ void k_energy(DevMesh m, EnergyArgs e) {
    const long x = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int K = e.K, M = e.M;
    if (x >= (long)m.N * M) return;
    const int i = (int)(x / M), mm = (int)(x - (long)i * M);
    const long KM = (long)K * M, K1M = (long)(K + 1) * M;
    int ed[6];
    double ck[6];
#pragma unroll
    for (int j = 0; j < 6; j++) {
        ed[j] = m.c_edge[6 * (long)i + j];
        ck[j] = m.c_ke[6 * (long)i + j];
    }
    auto kin = [&](int k) {
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < 6; j++) {
            if (ed[j] < 0) continue;
            const double uj = e.u[(long)ed[j] * KM + (long)k * M + mm];
            acc += ck[j] * (uj * uj);
        }
        return acc;
    };
    const double ps = e.ps[x];
    if (e.model == MODEL_SW) {
        const double b = e.b ? e.b[i] : 0.0;
        e.out[x] = ps * (kin(0) + e.grav * (0.5 * ps + b));
        return;
    }
    const double kappa = e.rd / e.cp, cv = e.cp - e.rd;
    double acc = 0.0;
    if (e.model == MODEL_HDC) {
        double phib = e.phis ? e.phis[i] : 0.0;
        for (int k = K - 1; k >= 0; k--) {
            const double dpi = (e.sig[k + 1] - e.sig[k]) * (ps - e.ptop);
            const double pit = e.ptop + e.sig[k] * (ps - e.ptop);
            const double pib = e.ptop + e.sig[k + 1] * (ps - e.ptop);
            const double pk = 0.5 * (pit + pib);
            const double T = e.Th[(long)i * KM + (long)k * M + mm] / dpi * pow(pk / e.p0, kappa);
            const double phit = phib + e.rd * T / pk * dpi;
            acc += dpi * (kin(k) + cv * T + 0.5 * (phit + phib));
            phib = phit;
        }
    } else {
        const double gamma = e.cp / cv;
        for (int k = 0; k < K; k++) {
            const double dpi = (e.sig[k + 1] - e.sig[k]) * (ps - e.ptop);
            const long t = (long)i * K1M + (long)k * M + mm, b = t + M;
            const double dphi = e.phi[t] - e.phi[b];
            const double pk = e.p0 * pow(e.rd * e.Th[(long)i * KM + (long)k * M + mm] / (e.p0 * dphi), gamma);
            const double T = pk * (dphi / dpi) / e.rd;
            const double kw = 0.25 * (e.w[t] * e.w[t] + e.w[b] * e.w[b]);
            acc += dpi * (kin(k) + kw + cv * T + 0.5 * (e.phi[t] + e.phi[b]));
        }
    }
    e.out[x] = acc / e.grav;
}

hipError_t launch_energy(const DevMesh &m, const EnergyArgs &e, hipStream_t s) {
    const long n = (long)m.N * e.M;
    hipLaunchKernelGGL(k_energy, dim3(nblocks(n, 256)), dim3(256), 0, s, m, e);
    return hipGetLastError();
}

// Hydrostatic column diagnostics of the stage's input state (ps_s, Th_s) in
// FP64 -- the formulas of cell_b's FP64 diagnostics (Eqs. 8-9): alpha = R_d T
// / p at the mid-layer pressure and the layer mean of the geopotential
// integrated upwards from phi_s -- for stages without forward-backward
// ordering.  One lane per (cell, member), levels in sequence.
__global__ void k_column_diag(StageArgs a) {
    const long x = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int K = a.K, M = a.M;
    if (x >= (long)a.mesh.N * M) return;
    const int i = (int)(x / M), mm = (int)(x - (long)i * M);
    const long KM = (long)K * M;
    const double ps = a.ps_s[x];
    double phib = a.phis[i];
    for (int k = K - 1; k >= 0; k--) {
        const long o = (long)i * KM + (long)k * M + mm;
        const double dpn = a.dsig[k] * (ps - a.ptop);
        const double pit = a.ptop + a.sig[k] * (ps - a.ptop);
        const double pib = a.ptop + a.sig[k + 1] * (ps - a.ptop);
        const double pk = 0.5 * (pit + pib);
        const double T = (a.Th_s[o] / dpn) * powpos(pk * a.inv_p0, a.kappa);
        const double al = a.rd * T / pk;
        const double phit = phib + al * dpn;
        a.alpha[o] = al;
        a.phim[o] = 0.5 * (phit + phib);
        phib = phit;
    }
}

hipError_t launch_column_diag(const StageArgs &a, hipStream_t s) {
    const long n = (long)a.mesh.N * a.M;
    hipLaunchKernelGGL(k_column_diag, dim3(nblocks(n, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_shadows(int model, const StageArgs &args, hipStream_t s) {
    StageArgs a = args;
    a.flat_block = 256;   // the kernel reads its work-group size from here
    const long n = (long)(a.mesh.E > a.mesh.N ? a.mesh.E : a.mesh.N) * a.K * a.M;
    if (model == MODEL_SW) hipLaunchKernelGGL(k_shadows<MODEL_SW>, dim3(nblocks(n, 256)), dim3(256), 0, s, a);
    else if (model == MODEL_HDC) hipLaunchKernelGGL(k_shadows<MODEL_HDC>, dim3(nblocks(n, 256)), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_shadows<MODEL_NDC>, dim3(nblocks(n, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// whether the non-hydrostatic surface geopotential varies (terrain)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) k_surface_check(const double *phi, long N, int K, int M, int *flag) {
    int any = 0;
    const long n = N * M, K1M = (long)(K + 1) * M;
    for (long x = threadIdx.x; x < n; x += blockDim.x) {
        const long i = x / M;
        const int mm = (int)(x - i * M);
        any |= phi[i * K1M + (long)K * M + mm] != phi[(long)K * M + mm];
    }
    any = __syncthreads_or(any);
    if (threadIdx.x == 0) flag[0] = any != 0;
}

hipError_t launch_surface_check(const double *phi, long N, int K, int M, int *flag, hipStream_t s) {
    hipLaunchKernelGGL(k_surface_check, dim3(1), dim3(1024), 0, s, phi, N, K, M, flag);
    return hipGetLastError();
}

}  // namespace mpdc
