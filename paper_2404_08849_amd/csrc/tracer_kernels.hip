// HIP kernels of the tracer transport and of the diagnostics for gfx950.
//
// Tracer transport (Eq. 10, horizontal part) with a third-order upwind flux
// and a Zalesak FCT limiter in each RK3 stage (Section 2.1); the layer-mass
// continuity uses the FP64 mass flux (Section 2.3).  Layout q[N][K][T]: one
// lane per (cell, level, tracer), tracer innermost, so the FP64 mass flux
// F[E][K] and the mesh tables are shared by the T lanes of a level.
// Three passes per stage, each cell-centric (every edge flux is formed by
// both of its cells, identically, so no edge array is written):
//   low     F^L = F q^n(upwind), q^td = [dpi q^n - dt_s D(F^L)]/dpi_new, and the
//           quadratic-fit second-derivative coefficients of q^(s-1)
//   limit   A = F q~ - F^L; bounds of {q^n, q^td} over the cell and its
//           neighbours; P+-, Q+-, R+-
//   update  C = min(R+ receiver, R- donor); q^(s) = [dpi q^n - dt_s D(F^L + C A)]/dpi_new
// R = double (all-FP64 policy) or float (mixed policy: q, fluxes and limiter
// in FP32, layer-mass continuity in FP64).  SG (the all-FP32 policy, float
// only): the layer-mass continuity too is FP32 -- the mass flux is read as an
// FP32 number everywhere and the new layer mass is formed in FP32.
#include <hip/hip_runtime.h>

#include <cfloat>

#include "dycore_kernels.h"

namespace mpdc {

template <typename R> __device__ __forceinline__ const R *tpick(const double *d, const float *f);
template <> __device__ __forceinline__ const double *tpick<double>(const double *d, const float *) { return d; }
template <> __device__ __forceinline__ const float *tpick<float>(const double *, const float *f) { return f; }

template <typename R> __device__ __forceinline__ R rinf();
template <> __device__ __forceinline__ double rinf<double>() { return __builtin_huge_val(); }
template <> __device__ __forceinline__ float rinf<float>() { return __builtin_huge_valf(); }

// a * b + c with one rounding (the library is built without FMA contraction)
__device__ __forceinline__ float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T, int L> struct alignas(sizeof(T) * L) TPack {
    T v[L];
};
template <typename T, int L> __device__ __forceinline__ TPack<T, L> tld(const T *p) {
    return *reinterpret_cast<const TPack<T, L> *>(p);
}
template <typename T, int L> __device__ __forceinline__ void tst(T *p, const TPack<T, L> &x) {
    *reinterpret_cast<TPack<T, L> *>(p) = x;
}
template <typename T> __device__ __forceinline__ void tld6(const T *p, T out[6]) {
    const TPack<T, 2> a = tld<T, 2>(p), b = tld<T, 2>(p + 2), c = tld<T, 2>(p + 4);
    out[0] = a.v[0]; out[1] = a.v[1]; out[2] = b.v[0]; out[3] = b.v[1]; out[4] = c.v[0]; out[5] = c.v[1];
}

// Slots per basic block of the tracer kernels' stencil loops (the gathers of
// a block are issued together), and whether a kernel reads the neighbour's
// q^n and second derivatives only where the neighbour is upwind (fewer bytes,
// but a wait per slot) -- both the fastest measured on MI355X (G8 x 30 x 8).
// A pentagon's pad slot (edge -1) is processed with edge 0, the cell itself
// as neighbour, zero flux and zero weights, so it adds nothing.
constexpr int kLowSlots = 3, kLimitSlots = 3, kUpdateSlots = 2;
constexpr bool kLimitUpwindLoads = false, kUpdateUpwindLoads = true;

// One lane = L consecutive tracers of one (cell, level).
struct TLane {
    int i, k, t0;
    long x;       // linear index of (i, k, t0)
    bool ok;
};
// UNI: one cell per work-group of exactly K T / L lanes; the cell, and so
// its stencil tables and its edges' tables, are the same in every lane, and
// the kernels read them with scalar loads.
template <int L, bool UNI> __device__ __forceinline__ TLane tracer_lane(const TracerArgs &a) {
    TLane r;
    const int lanes_k = a.T / L;
    if constexpr (UNI) {
        r.i = (int)xcd_block();
        r.ok = r.i < a.mesh.N;
        r.k = (int)threadIdx.x / lanes_k;
        r.t0 = ((int)threadIdx.x - r.k * lanes_k) * L;
        r.x = ((long)r.i * a.K + r.k) * a.T + r.t0;
        return r;
    }
    const int lanes = a.K * lanes_k;
    const long idx = (long)xcd_block() * a.cpb + threadIdx.x;   // a.cpb = threads per work-group
    r.ok = idx < (long)a.mesh.N * lanes;
    r.i = (int)(idx / lanes);
    const int rem = (int)(idx - (long)r.i * lanes);
    r.k = rem / lanes_k;
    r.t0 = (rem - r.k * lanes_k) * L;
    r.x = ((long)r.i * a.K + r.k) * a.T + r.t0;
    return r;
}

// Per-cell stencil shared by the three passes: edges, neighbours, outward
// signs via the divergence weights, the FP64 mass flux of each edge and the
// layer mass after this stage's FP64 continuity step.
template <typename R> struct Stencil {
    int ce[6], cn[6];
    R cdiv[6];
    double F[6];
    double dpi_n, dpin;
};
template <typename R, bool SG, bool UNI>
__device__ __forceinline__ void load_stencil(const TracerArgs &a, int i, int k, Stencil<R> &st) {
    const DevMesh &m = a.mesh;
    const long r6 = (long)i * kCellSlots;
    if constexpr (UNI) {
        sld6<int>(m.c_edge, r6, st.ce);
        sld6<int>(m.c_nbr, r6, st.cn);
        sld6<R>(tpick<R>(m.c_div, m.c_div32), r6, st.cdiv);
    } else {
        tld6<int>(m.c_edge + r6, st.ce);
        tld6<int>(m.c_nbr + r6, st.cn);
        tld6<R>(tpick<R>(m.c_div, m.c_div32) + r6, st.cdiv);
    }
    if constexpr (SG) {
        // all-FP32: the flux as an FP32 number, FP32 continuity
        float d = 0.0f;
#pragma unroll
        for (int s = 0; s < kCellSlots; s++) {
            const float f = (float)a.F[(long)(st.ce[s] < 0 ? 0 : st.ce[s]) * a.K + k];
            st.F[s] = (st.ce[s] >= 0) ? (double)f : 0.0;
            d = fmar((float)st.cdiv[s], (float)st.F[s], d);
        }
        const float dn = (float)a.dpi_n[(long)i * a.K + k];
        st.dpi_n = (double)dn;
        st.dpin = (double)(dn - (float)a.dts * d);
        return;
    }
    double c64[6];
    if constexpr (UNI) sld6<double>(m.c_div, r6, c64);
    else tld6<double>(m.c_div + r6, c64);
    double d = 0.0;
#pragma unroll
    for (int s = 0; s < kCellSlots; s++) {
        // a pentagon's pad slot reads edge 0 (no load under a condition) and
        // gets a zero flux
        const double f = a.F[(long)(st.ce[s] < 0 ? 0 : st.ce[s]) * a.K + k];
        st.F[s] = (st.ce[s] >= 0) ? f : 0.0;
        d += c64[s] * st.F[s];
    }
    st.dpi_n = a.dpi_n[(long)i * a.K + k];
    st.dpin = st.dpi_n - a.dts * d;
}

// Low-order (upwind) flux and antidiffusive flux A = F q~ - F^L of the edge in
// slot s of cell i, for L tracers.  q~ is the third-order upwind edge value of
// q_s: with the upwind weight 1 the two second-derivative terms reduce to
// -d^2/6 times the second derivative along the edge of the upwind cell alone,
// so only the upwind cell's q^n and second derivatives are used (the
// neighbour's are loaded either way: a load under a condition would cost a
// wait where the paths join).  The flux F_e is one FP64 number per
// edge-level, so the upwind cell is the same for the L tracers of a lane.
// qn_nb, if given, is q^n of the neighbour already loaded by the caller.
template <typename R, int L, bool UPWIND_LOADS, bool UNI>
__device__ __forceinline__ void edge_fluxes(const TracerArgs &a, const Stencil<R> &st, int s, int k, int t0,
                                            const R qn_i[L], const R qs_i[L], const R Hi[3][L],
                                            const TPack<R, L> *qn_nb, R FL[L], R Aa[L]) {
    const DevMesh &m = a.mesh;
    const int KT = a.K * a.T;
    const int e = st.ce[s] < 0 ? 0 : st.ce[s], nb = st.cn[s];   // pad slot: edge 0, the cell itself, F = 0
    const double Fd = st.F[s];
    const bool fwd = Fd >= 0.0;                              // c1 is upwind
    const bool up_self = fwd == (st.cdiv[s] > (R)0);
    const long on = (long)nb * KT + (long)k * a.T + t0;
    const TPack<R, L> qs_n = tld<R, L>((const R *)a.q_s + on);
    R qup[L], H0[L], H1[L], H2[L];
    const R *Hb = (const R *)a.hq + (long)nb * 3 * KT + (long)k * a.T + t0;
    if constexpr (UPWIND_LOADS) {
        // the neighbour's q^n and second derivatives only where it is upwind
        if (up_self) {
#pragma unroll
            for (int j = 0; j < L; j++) {
                qup[j] = qn_i[j];
                H0[j] = Hi[0][j];
                H1[j] = Hi[1][j];
                H2[j] = Hi[2][j];
            }
        } else {
            const TPack<R, L> qn_n = qn_nb ? *qn_nb : tld<R, L>((const R *)a.q_n + on);
            const TPack<R, L> h0 = tld<R, L>(Hb), h1 = tld<R, L>(Hb + KT), h2 = tld<R, L>(Hb + 2 * KT);
#pragma unroll
            for (int j = 0; j < L; j++) {
                qup[j] = qn_n.v[j];
                H0[j] = h0.v[j];
                H1[j] = h1.v[j];
                H2[j] = h2.v[j];
            }
        }
    } else {
        const TPack<R, L> qn_n = qn_nb ? *qn_nb : tld<R, L>((const R *)a.q_n + on);
        const TPack<R, L> h0 = tld<R, L>(Hb), h1 = tld<R, L>(Hb + KT), h2 = tld<R, L>(Hb + 2 * KT);
#pragma unroll
        for (int j = 0; j < L; j++) {
            qup[j] = up_self ? qn_i[j] : qn_n.v[j];
            H0[j] = up_self ? Hi[0][j] : h0.v[j];
            H1[j] = up_self ? Hi[1][j] : h1.v[j];
            H2[j] = up_self ? Hi[2][j] : h2.v[j];
        }
    }
    // the neighbour direction in the upwind cell's frame (c1: first triple)
    R d0, d1, d2, m2c;
    if constexpr (UNI) {
        // both triples by scalar loads (the edge is the same in every lane; the
        // upwind side depends on the level's flux)
        const R *hd = tpick<R>(m.e_hdir, m.e_hdir32);
        const long o = (long)e * 6;
        const R a0 = sld(hd, o), a1 = sld(hd, o + 1), a2 = sld(hd, o + 2);
        const R b0 = sld(hd, o + 3), b1 = sld(hd, o + 4), b2 = sld(hd, o + 5);
        d0 = fwd ? a0 : b0;
        d1 = fwd ? a1 : b1;
        d2 = fwd ? a2 : b2;
        m2c = (R)-2 * sld(tpick<R>(m.e_d2, m.e_d2_32), (long)e);
    } else {
        const R *dir = tpick<R>(m.e_hdir, m.e_hdir32) + (long)e * 6 + (fwd ? 0 : 3);
        d0 = dir[0];
        d1 = dir[1];
        d2 = dir[2];
        m2c = (R)-2 * tpick<R>(m.e_d2, m.e_d2_32)[e];
    }
    const R F = (R)Fd;
#pragma unroll
    for (int j = 0; j < L; j++) {
        const R h = fmar(H0[j], d0, fmar(H1[j], d1, H2[j] * d2));
        const R qe = fmar(m2c, h, (R)0.5 * (qs_i[j] + qs_n.v[j]));
        FL[j] = F * qup[j];
        Aa[j] = fmar(F, qe, -FL[j]);
    }
}

template <typename R, int L, bool SG, bool UNI>
__global__ void __launch_bounds__(kTracerThreads) k_tr_low(TracerArgs a) {
    const TLane ln = tracer_lane<L, UNI>(a);
    if (!ln.ok) return;
    const DevMesh &m = a.mesh;
    const int KT = a.K * a.T;
    const int i = ln.i, k = ln.k, t0 = ln.t0;
    Stencil<R> st;
    load_stencil<R, SG, UNI>(a, i, k, st);
    const R *qn = (const R *)a.q_n;
    const R *qs = (const R *)a.q_s;
    R ch[3][6];
    const R *chp = tpick<R>(m.c_hess, m.c_hess32);
    const long r18 = (long)i * 3 * kCellSlots;
    if constexpr (UNI) {
        sld6<R>(chp, r18, ch[0]);
        sld6<R>(chp, r18 + kCellSlots, ch[1]);
        sld6<R>(chp, r18 + 2 * kCellSlots, ch[2]);
    } else {
        tld6<R>(chp + r18, ch[0]);
        tld6<R>(chp + r18 + kCellSlots, ch[1]);
        tld6<R>(chp + r18 + 2 * kCellSlots, ch[2]);
    }
    const TPack<R, L> qni = tld<R, L>(qn + ln.x), qsi = tld<R, L>(qs + ln.x);
    R dL[L], h[3][L];
#pragma unroll
    for (int j = 0; j < L; j++) dL[j] = h[0][j] = h[1][j] = h[2][j] = 0;
#pragma unroll
    for (int s = 0; s < kCellSlots; s++) {
        if (s % kLowSlots == 0 && st.ce[s] < 0) continue;   // never taken: slots 0..4 always exist
        const long on = (long)st.cn[s] * KT + (long)k * a.T + t0;
        const TPack<R, L> qsn = tld<R, L>(qs + on), qnn = tld<R, L>(qn + on);
        const double Fd = st.F[s];
        const bool up_self = (Fd >= 0.0) == (st.cdiv[s] > (R)0);
#pragma unroll
        for (int j = 0; j < L; j++) {
            const R dq = qsn.v[j] - qsi.v[j];
            h[0][j] = fmar(ch[0][s], dq, h[0][j]);
            h[1][j] = fmar(ch[1][s], dq, h[1][j]);
            h[2][j] = fmar(ch[2][s], dq, h[2][j]);
            dL[j] = fmar(st.cdiv[s], (R)Fd * (up_self ? qni.v[j] : qnn.v[j]), dL[j]);
        }
    }
    R *H = (R *)a.hq + (long)i * 3 * KT + (long)k * a.T + t0;
    TPack<R, L> p0, p1, p2, qt;
#pragma unroll
    for (int j = 0; j < L; j++) {
        p0.v[j] = h[0][j];
        p1.v[j] = h[1][j];
        p2.v[j] = h[2][j];
        qt.v[j] = ((R)st.dpi_n * qni.v[j] - (R)a.dts * dL[j]) / (R)st.dpin;
    }
    tst<R, L>(H, p0);
    tst<R, L>(H + KT, p1);
    tst<R, L>(H + 2 * KT, p2);
    tst<R, L>((R *)a.qtd + ln.x, qt);
}

template <typename R, int L>
__device__ __forceinline__ void load_own(const TracerArgs &a, const TLane &ln, R qn_i[L], R qs_i[L], R Hi[3][L]) {
    const int KT = a.K * a.T;
    const TPack<R, L> qn = tld<R, L>((const R *)a.q_n + ln.x), qs = tld<R, L>((const R *)a.q_s + ln.x);
    const R *Hb = (const R *)a.hq + (long)ln.i * 3 * KT + (long)ln.k * a.T + ln.t0;
    const TPack<R, L> h0 = tld<R, L>(Hb), h1 = tld<R, L>(Hb + KT), h2 = tld<R, L>(Hb + 2 * KT);
#pragma unroll
    for (int j = 0; j < L; j++) {
        qn_i[j] = qn.v[j];
        qs_i[j] = qs.v[j];
        Hi[0][j] = h0.v[j];
        Hi[1][j] = h1.v[j];
        Hi[2][j] = h2.v[j];
    }
}

template <typename R, int L, bool SG, bool UNI>
__global__ void __launch_bounds__(kTracerThreads) k_tr_limit(TracerArgs a) {
    const TLane ln = tracer_lane<L, UNI>(a);
    if (!ln.ok) return;
    const int KT = a.K * a.T;
    const int i = ln.i, k = ln.k, t0 = ln.t0;
    Stencil<R> st;
    load_stencil<R, SG, UNI>(a, i, k, st);
    R qn_i[L], qs_i[L], Hi[3][L];
    load_own<R, L>(a, ln, qn_i, qs_i, Hi);
    const R *qn = (const R *)a.q_n;
    const R *qtd = (const R *)a.qtd;
    const TPack<R, L> qti = tld<R, L>(qtd + ln.x);
    R qmax[L], qmin[L], Pp[L], Pm[L];
#pragma unroll
    for (int j = 0; j < L; j++) {
        qmax[j] = qn_i[j] > qti.v[j] ? qn_i[j] : qti.v[j];
        qmin[j] = qn_i[j] < qti.v[j] ? qn_i[j] : qti.v[j];
        Pp[j] = Pm[j] = 0;
    }
#pragma unroll
    for (int s = 0; s < kCellSlots; s++) {
        if (s % kLimitSlots == 0 && st.ce[s] < 0) continue;
        const long on = (long)st.cn[s] * KT + (long)k * a.T + t0;
        const TPack<R, L> qnn = tld<R, L>(qn + on), qtn = tld<R, L>(qtd + on);
        R FL[L], Aa[L];
        edge_fluxes<R, L, kLimitUpwindLoads, UNI>(a, st, s, k, t0, qn_i, qs_i, Hi, &qnn, FL, Aa);
#pragma unroll
        for (int j = 0; j < L; j++) {
            qmax[j] = fmax(qmax[j], fmax(qnn.v[j], qtn.v[j]));
            qmin[j] = fmin(qmin[j], fmin(qnn.v[j], qtn.v[j]));
            const R fo = st.cdiv[s] * Aa[j];
            if (fo < (R)0) Pp[j] -= fo;
            if (fo > (R)0) Pm[j] += fo;
        }
    }
    const R rdt = (R)(st.dpin / a.dts);
    TPack<R, L> rp, rm;
#pragma unroll
    for (int j = 0; j < L; j++) {
        if (!a.fct) {
            qmax[j] = rinf<R>();
            qmin[j] = -rinf<R>();
        }
        const R Qp = (qmax[j] - qti.v[j]) * rdt, Qm = (qti.v[j] - qmin[j]) * rdt;
        rp.v[j] = (Pp[j] > (R)0) ? fmin((R)1, Qp / Pp[j]) : (R)0;
        rm.v[j] = (Pm[j] > (R)0) ? fmin((R)1, Qm / Pm[j]) : (R)0;
    }
    tst<R, L>((R *)a.rp + ln.x, rp);
    tst<R, L>((R *)a.rm + ln.x, rm);
}

template <typename R, int L, bool SG, bool UNI>
__global__ void __launch_bounds__(kTracerThreads) k_tr_update(TracerArgs a) {
    const TLane ln = tracer_lane<L, UNI>(a);
    if (!ln.ok) return;
    const int KT = a.K * a.T;
    const int i = ln.i, k = ln.k, t0 = ln.t0;
    Stencil<R> st;
    load_stencil<R, SG, UNI>(a, i, k, st);
    R qn_i[L], qs_i[L], Hi[3][L];
    load_own<R, L>(a, ln, qn_i, qs_i, Hi);
    const R *rp = (const R *)a.rp;
    const R *rm = (const R *)a.rm;
    const TPack<R, L> rpi = tld<R, L>(rp + ln.x), rmi = tld<R, L>(rm + ln.x);
    R dT[L];
#pragma unroll
    for (int j = 0; j < L; j++) dT[j] = 0;
#pragma unroll
    for (int s = 0; s < kCellSlots; s++) {
        if (s % kUpdateSlots == 0 && st.ce[s] < 0) continue;
        const long on = (long)st.cn[s] * KT + (long)k * a.T + t0;
        const TPack<R, L> rpn = tld<R, L>(rp + on), rmn = tld<R, L>(rm + on);
        R FL[L], Aa[L];
        edge_fluxes<R, L, kUpdateUpwindLoads, UNI>(a, st, s, k, t0, qn_i, qs_i, Hi, nullptr, FL, Aa);
        const bool self_c1 = st.cdiv[s] > (R)0;
#pragma unroll
        for (int j = 0; j < L; j++) {
            const R rp1 = self_c1 ? rpi.v[j] : rpn.v[j], rp2 = self_c1 ? rpn.v[j] : rpi.v[j];
            const R rm1 = self_c1 ? rmi.v[j] : rmn.v[j], rm2 = self_c1 ? rmn.v[j] : rmi.v[j];
            const R C = (Aa[j] >= (R)0) ? fmin(rp2, rm1) : fmin(rp1, rm2);
            dT[j] = fmar(st.cdiv[s], fmar(C, Aa[j], FL[j]), dT[j]);
        }
    }
    TPack<R, L> qo;
#pragma unroll
    for (int j = 0; j < L; j++) qo.v[j] = ((R)st.dpi_n * qn_i[j] - (R)a.dts * dT[j]) / (R)st.dpin;
    tst<R, L>((R *)a.q_o + ln.x, qo);
    if (a.last_stage && t0 == 0) a.dpi_o[(long)i * a.K + k] = st.dpin;
}

namespace {
inline unsigned tblocks(long n, int b) { return (unsigned)((n + b - 1) / b); }
template <typename R, int L, bool SG>
hipError_t launch_tr_l(const TracerArgs &a, int which, hipStream_t s) {
    if (a.cpb == 1) {
        // one cell per work-group (K T / L <= 512 threads, checked by the host)
        const unsigned nb = a.mesh.N;
        const int b = a.K * (a.T / L);
        switch (which) {
        case TKERNEL_LOW: hipLaunchKernelGGL((k_tr_low<R, L, SG, true>), dim3(nb), dim3(b), 0, s, a); break;
        case TKERNEL_LIMIT: hipLaunchKernelGGL((k_tr_limit<R, L, SG, true>), dim3(nb), dim3(b), 0, s, a); break;
        case TKERNEL_UPDATE: hipLaunchKernelGGL((k_tr_update<R, L, SG, true>), dim3(nb), dim3(b), 0, s, a); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    const long n = (long)a.mesh.N * a.K * (a.T / L);
    TracerArgs ab = a;
    ab.cpb = a.cpb > 0 ? a.cpb : 256;   // the kernels read the work-group size from here
    const int b = ab.cpb;
    switch (which) {
    case TKERNEL_LOW: hipLaunchKernelGGL((k_tr_low<R, L, SG, false>), dim3(tblocks(n, b)), dim3(b), 0, s, ab); break;
    case TKERNEL_LIMIT: hipLaunchKernelGGL((k_tr_limit<R, L, SG, false>), dim3(tblocks(n, b)), dim3(b), 0, s, ab); break;
    case TKERNEL_UPDATE: hipLaunchKernelGGL((k_tr_update<R, L, SG, false>), dim3(tblocks(n, b)), dim3(b), 0, s, ab); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
template <typename R, bool SG>
hipError_t launch_tr(const TracerArgs &a, int which, hipStream_t s) {
    if constexpr (sizeof(R) == 4)
        if (a.vpl == 8) return launch_tr_l<R, 8, SG>(a, which, s);
    if (a.vpl == 4) return launch_tr_l<R, 4, SG>(a, which, s);
    if (a.vpl == 2) return launch_tr_l<R, 2, SG>(a, which, s);
    return launch_tr_l<R, 1, SG>(a, which, s);
}
}  // namespace

hipError_t launch_tracer_kernel(int policy, const TracerArgs &a, int which, hipStream_t s) {
    if (policy == POLICY_DBL) return launch_tr<double, false>(a, which, s);
    if (policy == POLICY_SGL) return launch_tr<float, true>(a, which, s);
    return launch_tr<float, false>(a, which, s);
}

// ---------------------------------------------------------------------------
// vertical step (Eq. 10, the vertical flux divergence), time-split after the
// horizontal stages: adaptively implicit first-order upwind
// ---------------------------------------------------------------------------
// Interface k (0..K) lies between layers k-1 and k; vflux[i][k] is the mass
// flux through it, positive towards the surface (the lid and surface values
// are taken as zero).  New layer mass: dpi_k - dt (m_{k+1} - m_k).  Each flux
// splits into an explicit part, capped at a Courant number of 1/2 with respect
// to its donor layer (so the explicit update alone is monotone), and the
// implicit remainder; both are first-order upwind, the implicit part with the
// new mixing ratio:
//   dpi_new_k q_k + dt (GI_{k+1} - GI_k) = dpi_k qh_k - dt (GE_{k+1} - GE_k).
// The tridiagonal matrix is an M-matrix (new q is a convex combination of the
// old values) and the same for every tracer of a column.  A work-group holds
// whole columns: it stages their q, layer masses and fluxes in LDS with
// coalesced loads, one lane per (cell, tracer) runs the Thomas algorithm down
// its column in FP64 on LDS (the column's tracer-0 lane keeps the shared
// elimination factors), and the results go back with coalesced stores; q and
// dpi are updated in place.
constexpr int kVertThreads = 512;
__host__ __device__ inline long vert_column_doubles(int K, int T) { return (long)K * T + 3L * K + 1; }

// dst[x] = src[x] for x < n by all nthr threads of the work-group, eight loads
// in flight per thread (clamped indices, so none sits under a condition)
template <typename S>
__device__ __forceinline__ void stage_in(double *dst, const S *src, long n, int tid, int nthr) {
    constexpr int U = 8;
    for (long b = tid; b < n; b += (long)U * nthr) {
        S v[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const long x = b + (long)u * nthr;
            v[u] = src[x < n ? x : n - 1];
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const long x = b + (long)u * nthr;
            if (x < n) dst[x] = (double)v[u];
        }
    }
}

template <typename R>
__global__ void __launch_bounds__(kVertThreads) k_tr_vert(TracerArgs a, int cols) {
    extern __shared__ double vlds[];
    const int K = a.K, T = a.T;
    const int tid = threadIdx.x, nthr = cols * T;
    const long i0 = (long)blockIdx.x * cols;
    const int ncol = (int)(a.mesh.N - i0 < cols ? a.mesh.N - i0 : cols);
    double *sq = vlds;                            // [cols][K][T]: q^h, then the forward factors, then q
    double *sd = sq + (long)cols * K * T;         // [cols][K]: layer masses
    double *sm = sd + (long)cols * K;             // [cols][K+1]: interface fluxes
    double *sc = sm + (long)cols * (K + 1);       // [cols][K]: elimination factors (shared by the tracers)
    R *q = (R *)a.q_o;
    double *dpi = a.dpi_o;
    const double dt = a.dts, half_over_dt = 0.5 / a.dts;
    const long nq = (long)ncol * K * T, nd = (long)ncol * K, nm = (long)ncol * (K + 1);
    stage_in<R>(sq, q + i0 * K * T, nq, tid, nthr);
    stage_in<double>(sd, dpi + i0 * K, nd, tid, nthr);
    stage_in<double>(sm, a.vflux + i0 * (K + 1), nm, tid, nthr);
    __syncthreads();
    const int lc = tid / T, t = tid - lc * T;
    const bool valid = lc < ncol;
    if (valid) {
        double *qc = sq + (long)lc * K * T + t;
        const double *dh = sd + (long)lc * K, *mc = sm + (long)lc * (K + 1);
        double *cf = sc + (long)lc * K;
        double mEt = 0.0, aIt = 0.0;       // top interface of layer k: explicit flux, dt * implicit flux
        double qu = 0.0;                   // q^h of the layer above
        double qk = qc[0];
        double cprev = 0.0, dprev = 0.0;
        for (int k = 0; k < K; k++) {
            const bool below = k < K - 1;
            const int kn = below ? k + 1 : k;   // clamped: the surface interface carries no flux
            const double mb = below ? mc[k + 1] : 0.0;
            const double mt = k > 0 ? mc[k] : 0.0;
            const double dk = dh[k], dn = dh[kn];
            const double qd = qc[(long)kn * T];
            // explicit part: the flux capped at half the donor's mass per dt
            // (Courant number 1/2), with the flux's sign
            const double cap = half_over_dt * (mb >= 0.0 ? dk : dn);
            const double mEb = fabs(mb) > cap ? copysign(cap, mb) : mb;
            const double aIb = dt * (mb - mEb);
            const double dnew = dk - dt * (mb - mt);
            const double sub = -fmax(aIt, 0.0);
            const double dia = dnew + fmax(aIb, 0.0) + fmax(-aIt, 0.0);
            const double sup = -fmax(-aIb, 0.0);
            const double get = mEt * (mEt >= 0.0 ? qu : qk);   // zero at the lid (mEt = 0)
            const double geb = mEb * (mEb >= 0.0 ? qk : qd);   // zero at the surface
            const double rhs = dk * qk - dt * (geb - get);
            const double rden = 1.0 / (dia - sub * cprev);
            cprev = below ? sup * rden : 0.0;
            dprev = (rhs - sub * dprev) * rden;
            if (t == 0) cf[k] = cprev;
            qc[(long)k * T] = dprev;           // q^h of layer k is no longer needed (qu holds it)
            mEt = mEb;
            aIt = aIb;
            qu = qk;
            qk = qd;
        }
    }
    __syncthreads();
    if (valid) {
        double *qc = sq + (long)lc * K * T + t;
        const double *cf = sc + (long)lc * K;
        double x = 0.0;
        for (int k = K - 1; k >= 0; k--) {
            x = qc[(long)k * T] - cf[k] * x;
            qc[(long)k * T] = x;
        }
    }
    // new layer masses (every lane of the group has read them above)
    for (long x = tid; x < nd; x += nthr) {
        const int c = (int)(x / K), k = (int)(x - (long)c * K);
        const double *mc = sm + (long)c * (K + 1);
        const double mb = k < K - 1 ? mc[k + 1] : 0.0, mt = k > 0 ? mc[k] : 0.0;
        dpi[i0 * K + x] = sd[x] - dt * (mb - mt);
    }
    __syncthreads();
    for (long x = tid; x < nq; x += nthr) q[i0 * K * T + x] = (R)sq[x];   // (stores: no waits)
}

int tracer_vert_columns(int K, int T) {
    const long per = vert_column_doubles(K, T) * 8;
    if (per > 65536 || T > kVertThreads) return 0;   // one column must fit the LDS of a work-group
    int c = kVertThreads / T;
    while (c > 1 && (long)c * per > 32768) c--;
    return c;
}

hipError_t launch_tracer_vertical(int policy, const TracerArgs &a, hipStream_t s) {
    const int cols = tracer_vert_columns(a.K, a.T);
    if (cols < 1) return hipErrorInvalidValue;
    const unsigned nb = (unsigned)((a.mesh.N + cols - 1) / cols);
    const size_t lds = (size_t)cols * vert_column_doubles(a.K, a.T) * 8;
    if (policy == POLICY_DBL)
        hipLaunchKernelGGL(k_tr_vert<double>, dim3(nb), dim3(cols * a.T), lds, s, a, cols);
    else
        hipLaunchKernelGGL(k_tr_vert<float>, dim3(nb), dim3(cols * a.T), lds, s, a, cols);
    return hipGetLastError();
}

// the dycore's accumulated mass fluxes, averaged over its n steps, become the
// tracer's FP64 fluxes; the accumulators restart from zero
__global__ void k_couple(double *Facc, double *Macc, double *F, double *vflux, long nF, long nM, double n) {
    const long x = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x < nF) {
        F[x] = Facc[x] / n;
        Facc[x] = 0.0;
    }
    if (x < nM) {
        vflux[x] = Macc[x] / n;
        Macc[x] = 0.0;
    }
}

hipError_t launch_couple(double *Facc, double *Macc, double *F, double *vflux, long nF, long nM, long n,
                         hipStream_t s) {
    const long m = nF > nM ? nF : nM;
    hipLaunchKernelGGL(k_couple, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, Facc, Macc, F, vflux, nF, nM,
                       (double)n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// diagnostics: per-block FP64 partial sums in a fixed order (no atomics)
// partial[b] = {sum A (x-off) w, min x, max x, sum A|x-r|, sum A|r|,
//               sum A (x-r)^2, sum A r^2, max|x-r|, max|r|}
// ---------------------------------------------------------------------------
constexpr int kDiagThreads = 256;
constexpr int kDiagVals = 9;

__global__ void __launch_bounds__(kDiagThreads) k_diag(DiagArgs a) {
    __shared__ double s[kDiagVals][kDiagThreads];
    double acc[kDiagVals] = {0.0, __builtin_huge_val(), -__builtin_huge_val(), 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const long total = a.n * a.inner;
    for (long idx = (long)blockIdx.x * kDiagThreads + threadIdx.x; idx < total; idx += (long)gridDim.x * kDiagThreads) {
        const long i = idx / a.inner;
        const double A = a.area ? a.area[i] : 1.0;
        const long xi = idx * a.xs + a.xo;
        const double x = a.x ? a.x[xi] : (double)a.x32[xi];
        const double wv = a.w ? a.w[idx] : 1.0;
        acc[0] += A * (x - a.offset) * wv;
        acc[1] = fmin(acc[1], x);
        acc[2] = fmax(acc[2], x);
        if (a.ref) {
            const double r = a.ref[xi];
            const double d = x - r;
            acc[3] += A * fabs(d);
            acc[4] += A * fabs(r);
            acc[5] += A * d * d;
            acc[6] += A * r * r;
            acc[7] = fmax(acc[7], fabs(d));
            acc[8] = fmax(acc[8], fabs(r));
        }
    }
    for (int v = 0; v < kDiagVals; v++) s[v][threadIdx.x] = acc[v];
    __syncthreads();
    for (int h = kDiagThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            const int o = threadIdx.x + h;
            s[0][threadIdx.x] += s[0][o];
            s[1][threadIdx.x] = fmin(s[1][threadIdx.x], s[1][o]);
            s[2][threadIdx.x] = fmax(s[2][threadIdx.x], s[2][o]);
            for (int v = 3; v < 7; v++) s[v][threadIdx.x] += s[v][o];
            s[7][threadIdx.x] = fmax(s[7][threadIdx.x], s[7][o]);
            s[8][threadIdx.x] = fmax(s[8][threadIdx.x], s[8][o]);
        }
        __syncthreads();
    }
    if (threadIdx.x < kDiagVals) a.partial[(long)blockIdx.x * kDiagVals + threadIdx.x] = s[threadIdx.x][0];
}

__global__ void __launch_bounds__(kDiagThreads) k_nonfinite(const double *x, const float *x32, long n,
                                                            unsigned long long *partial) {
    __shared__ unsigned long long s[kDiagThreads];
    unsigned long long c = 0;
    for (long idx = (long)blockIdx.x * kDiagThreads + threadIdx.x; idx < n; idx += (long)gridDim.x * kDiagThreads) {
        const double v = x ? x[idx] : (double)x32[idx];
        if (!isfinite(v)) c++;
    }
    s[threadIdx.x] = c;
    __syncthreads();
    for (int h = kDiagThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = s[0];
}

hipError_t launch_diag(const DiagArgs &a, int nblocks, hipStream_t s) {
    hipLaunchKernelGGL(k_diag, dim3(nblocks), dim3(kDiagThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_nonfinite(const double *x, const float *x32, long n, unsigned long long *partial, int nblocks,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_nonfinite, dim3(nblocks), dim3(kDiagThreads), 0, s, x, x32, n, partial);
    return hipGetLastError();
}

// largest advective Courant number max |u_e| dt / d_e over the edge field
// u [E][inner]; per-block maxima (a NaN anywhere gives a NaN maximum)
__global__ void __launch_bounds__(kDiagThreads) k_cfl(const double *u, const double *dinv, long E, long inner,
                                                      double dt, double *partial) {
    __shared__ double s[kDiagThreads];
    double c = 0.0;
    for (long idx = (long)blockIdx.x * kDiagThreads + threadIdx.x; idx < E * inner; idx += (long)gridDim.x * kDiagThreads) {
        const double v = fabs(u[idx]) * dt * dinv[idx / inner];
        c = (v > c || v != v) ? v : c;
    }
    s[threadIdx.x] = c;
    __syncthreads();
    for (int h = kDiagThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            const double o = s[threadIdx.x + h];
            if (o > s[threadIdx.x] || o != o) s[threadIdx.x] = o;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = s[0];
}

hipError_t launch_cfl(const double *u, const double *dinv, long E, long inner, double dt, double *partial,
                      int nblocks, hipStream_t s) {
    hipLaunchKernelGGL(k_cfl, dim3(nblocks), dim3(kDiagThreads), 0, s, u, dinv, E, inner, dt, partial);
    return hipGetLastError();
}

}  // namespace mpdc
