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
// in FP32, layer-mass continuity in FP64).
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

struct TIdx {
    int i, k, t;
    long x;       // (i, k, t) linear index
    bool ok;
};

__device__ __forceinline__ TIdx tracer_index(const TracerArgs &a) {
    TIdx r;
    const int KT = a.K * a.T;
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    r.ok = idx < (long)a.mesh.N * KT;
    r.i = (int)(idx / KT);
    const int kt = (int)(idx - (long)r.i * KT);
    r.k = kt / a.T;
    r.t = kt - r.k * a.T;
    r.x = idx;
    return r;
}

// divergence of the FP64 mass flux at (i, k): sum_j s l F / A
__device__ __forceinline__ double div_F(const TracerArgs &a, int i, int k) {
    const DevMesh &m = a.mesh;
    double d = 0.0;
#pragma unroll
    for (int j = 0; j < kCellSlots; j++) {
        const int e = m.c_edge[(long)i * kCellSlots + j];
        if (e < 0) continue;
        d += m.c_div[(long)i * kCellSlots + j] * a.F[(long)e * a.K + k];
    }
    return d;
}

// low-order (upwind) flux and antidiffusive flux A = F q~ - F^L of edge e,
// seen from cell i (slot j).  q~ is the third-order upwind edge value of q_s.
template <typename R>
__device__ __forceinline__ void edge_fluxes(const TracerArgs &a, int i, int e, int nb, int k, int t, R &FL, R &Aa) {
    const DevMesh &m = a.mesh;
    const int KT = a.K * a.T;
    const R *qn = (const R *)a.q_n;
    const R *qs = (const R *)a.q_s;
    const R *H = (const R *)a.hq;
    const int side = (m.e_cell[2 * (long)e] == i) ? 0 : 1;
    const int c1 = side ? nb : i, c2 = side ? i : nb;
    const double Fd = a.F[(long)e * a.K + k];
    const R F = (R)Fd;
    const long o1 = (long)c1 * KT + (long)k * a.T + t, o2 = (long)c2 * KT + (long)k * a.T + t;
    FL = F * ((Fd >= 0.0) ? qn[o1] : qn[o2]);
    const R *hdir = tpick<R>(m.e_hdir, m.e_hdir32) + (long)e * 6;
    const long h1 = (long)c1 * 3 * KT + (long)k * a.T + t, h2 = (long)c2 * 3 * KT + (long)k * a.T + t;
    const R q1d = H[h1] * hdir[0] + H[h1 + KT] * hdir[1] + H[h1 + 2 * KT] * hdir[2];
    const R q2d = H[h2] * hdir[3] + H[h2 + KT] * hdir[4] + H[h2 + 2 * KT] * hdir[5];
    const R c = tpick<R>(m.e_d2, m.e_d2_32)[e];
    const R sg = (Fd >= 0.0) ? (R)1 : (R)-1;
    const R qe = (R)0.5 * (qs[o1] + qs[o2]) - c * (q1d + q2d) + sg * c * (q2d - q1d);
    Aa = F * qe - FL;
}

template <typename R>
__global__ void __launch_bounds__(1024) k_tr_low(TracerArgs a) {
    const TIdx ix = tracer_index(a);
    if (!ix.ok) return;
    const DevMesh &m = a.mesh;
    const int KT = a.K * a.T;
    const int i = ix.i, k = ix.k, t = ix.t;
    const R *qn = (const R *)a.q_n;
    const R *qs = (const R *)a.q_s;
    const R *cdiv = tpick<R>(m.c_div, m.c_div32) + (long)i * kCellSlots;
    const R *ch = tpick<R>(m.c_hess, m.c_hess32) + (long)i * 3 * kCellSlots;
    const double dpi_n = a.dpi_n[(long)i * a.K + k];
    const double dpin = dpi_n - a.dts * div_F(a, i, k);
    const R qni = qn[ix.x], qsi = qs[ix.x];
    R dL = 0, h0 = 0, h1 = 0, h2 = 0;
#pragma unroll
    for (int j = 0; j < kCellSlots; j++) {
        const int nb = m.c_nbr[(long)i * kCellSlots + j];
        const long on = (long)nb * KT + (long)k * a.T + t;
        const R dq = qs[on] - qsi;
        h0 += ch[j] * dq;
        h1 += ch[kCellSlots + j] * dq;
        h2 += ch[2 * kCellSlots + j] * dq;
        const int e = m.c_edge[(long)i * kCellSlots + j];
        if (e < 0) continue;
        const double Fd = a.F[(long)e * a.K + k];
        const bool up_self = (Fd >= 0.0) == (m.e_cell[2 * (long)e] == i);
        dL += cdiv[j] * ((R)Fd * (up_self ? qni : qn[on]));
    }
    R *H = (R *)a.hq + (long)i * 3 * KT + (long)k * a.T + t;
    H[0] = h0;
    H[KT] = h1;
    H[2 * KT] = h2;
    ((R *)a.qtd)[ix.x] = ((R)dpi_n * qni - (R)a.dts * dL) / (R)dpin;
}

template <typename R>
__global__ void __launch_bounds__(1024) k_tr_limit(TracerArgs a) {
    const TIdx ix = tracer_index(a);
    if (!ix.ok) return;
    const DevMesh &m = a.mesh;
    const int KT = a.K * a.T;
    const int i = ix.i, k = ix.k, t = ix.t;
    const R *qn = (const R *)a.q_n;
    const R *qtd = (const R *)a.qtd;
    const R *cdiv = tpick<R>(m.c_div, m.c_div32) + (long)i * kCellSlots;
    const double dpin = a.dpi_n[(long)i * a.K + k] - a.dts * div_F(a, i, k);
    const R qtdi = qtd[ix.x];
    R qmax = qn[ix.x] > qtdi ? qn[ix.x] : qtdi;
    R qmin = qn[ix.x] < qtdi ? qn[ix.x] : qtdi;
    R Pp = 0, Pm = 0;
#pragma unroll
    for (int j = 0; j < kCellSlots; j++) {
        const int e = m.c_edge[(long)i * kCellSlots + j];
        if (e < 0) continue;
        const int nb = m.c_nbr[(long)i * kCellSlots + j];
        const long on = (long)nb * KT + (long)k * a.T + t;
        qmax = fmax(qmax, fmax(qn[on], qtd[on]));
        qmin = fmin(qmin, fmin(qn[on], qtd[on]));
        R FL, Aa;
        edge_fluxes<R>(a, i, e, nb, k, t, FL, Aa);
        const R fo = cdiv[j] * Aa;
        if (fo < (R)0) Pp -= fo;
        if (fo > (R)0) Pm += fo;
    }
    if (!a.fct) {
        qmax = rinf<R>();
        qmin = -rinf<R>();
    }
    const R rdt = (R)(dpin / a.dts);
    const R Qp = (qmax - qtdi) * rdt, Qm = (qtdi - qmin) * rdt;
    ((R *)a.rp)[ix.x] = (Pp > (R)0) ? fmin((R)1, Qp / Pp) : (R)0;
    ((R *)a.rm)[ix.x] = (Pm > (R)0) ? fmin((R)1, Qm / Pm) : (R)0;
}

template <typename R>
__global__ void __launch_bounds__(1024) k_tr_update(TracerArgs a) {
    const TIdx ix = tracer_index(a);
    if (!ix.ok) return;
    const DevMesh &m = a.mesh;
    const int KT = a.K * a.T;
    const int i = ix.i, k = ix.k, t = ix.t;
    const R *qn = (const R *)a.q_n;
    const R *rp = (const R *)a.rp;
    const R *rm = (const R *)a.rm;
    const R *cdiv = tpick<R>(m.c_div, m.c_div32) + (long)i * kCellSlots;
    const double dpi_n = a.dpi_n[(long)i * a.K + k];
    const double dpin = dpi_n - a.dts * div_F(a, i, k);
    R dT = 0;
#pragma unroll
    for (int j = 0; j < kCellSlots; j++) {
        const int e = m.c_edge[(long)i * kCellSlots + j];
        if (e < 0) continue;
        const int nb = m.c_nbr[(long)i * kCellSlots + j];
        R FL, Aa;
        edge_fluxes<R>(a, i, e, nb, k, t, FL, Aa);
        const bool self_c1 = (m.e_cell[2 * (long)e] == i);
        const long oi = ix.x, on = (long)nb * KT + (long)k * a.T + t;
        const long o1 = self_c1 ? oi : on, o2 = self_c1 ? on : oi;
        const R C = (Aa >= (R)0) ? fmin(rp[o2], rm[o1]) : fmin(rp[o1], rm[o2]);
        dT += cdiv[j] * (FL + C * Aa);
    }
    ((R *)a.q_o)[ix.x] = ((R)dpi_n * qn[ix.x] - (R)a.dts * dT) / (R)dpin;
    if (a.last_stage && t == 0) a.dpi_o[(long)i * a.K + k] = dpin;
}

namespace {
inline unsigned tblocks(long n, int b) { return (unsigned)((n + b - 1) / b); }
template <typename R>
hipError_t launch_tr(const TracerArgs &a, int which, hipStream_t s) {
    const long n = (long)a.mesh.N * a.K * a.T;
    const int b = a.cpb > 0 ? a.cpb : 256;
    switch (which) {
    case TKERNEL_LOW: hipLaunchKernelGGL(k_tr_low<R>, dim3(tblocks(n, b)), dim3(b), 0, s, a); break;
    case TKERNEL_LIMIT: hipLaunchKernelGGL(k_tr_limit<R>, dim3(tblocks(n, b)), dim3(b), 0, s, a); break;
    case TKERNEL_UPDATE: hipLaunchKernelGGL(k_tr_update<R>, dim3(tblocks(n, b)), dim3(b), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
}  // namespace

hipError_t launch_tracer_kernel(int policy, const TracerArgs &a, int which, hipStream_t s) {
    return policy == POLICY_DBL ? launch_tr<double>(a, which, s) : launch_tr<float>(a, which, s);
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

}  // namespace mpdc
