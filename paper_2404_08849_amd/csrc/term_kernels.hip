// Per-term precision engine of the hydrostatic dycore, for the iterative
// precision reduction of Section 2.2 (Eqs. 1-2): an RK stage as a chain of
// unfused kernels, one per term of the continuity, theta_m and momentum
// equations (Eqs. 3-5) and of the column diagnostics (Eqs. 8-9).  Each kernel
// is built in FP32 and in FP64, and a bit of the state's term mask picks the
// precision of each term.  A term computed in FP32 takes its FP64 inputs
// rounded to FP32 (as the mixed kernels read FP32 shadows) and its result is
// kept in FP64 storage, rounded from the FP32 value; the prognostic state is
// FP64 and is updated in FP64.  With no bit set this is a plain FP64
// implementation of the stage (checked against the oracle); the bits of the
// mixed policy's FP32 terms give its split.  One member (M = 1), layout
// [entity][K], one lane per entity-level (column kernels: per cell).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "dycore_kernels.h"

namespace mpdc {
namespace {

template <typename T> __device__ __forceinline__ const T *tb(const double *d, const float *f);
template <> __device__ __forceinline__ const double *tb<double>(const double *d, const float *) { return d; }
template <> __device__ __forceinline__ const float *tb<float>(const double *, const float *f) { return f; }

__device__ __forceinline__ double tpow(double x, double y) { return exp(y * log(x)); }
__device__ __forceinline__ float tpow(float x, float y) { return expf(y * logf(x)); }

inline unsigned tgrid(long n) { return (unsigned)((n + 255) / 256); }

__device__ __forceinline__ double layer_mass(const StageArgs &a, int k, double ps) { return a.dsig[k] * (ps - a.ptop); }

// mass flux F = dpi_e u, dpi_e the mean layer mass of the edge's cells (Eq. 3)
template <typename T> __global__ void k_t_flux(StageArgs a, TermArgs x) {
    const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int K = a.K;
    if (id >= (long)a.mesh.E * K) return;
    const int e = (int)(id / K), k = (int)(id - (long)e * K);
    const int c1 = a.mesh.e_cell[2 * e], c2 = a.mesh.e_cell[2 * e + 1];
    const double dpe = 0.5 * (layer_mass(a, k, a.ps_s[c1]) + layer_mass(a, k, a.ps_s[c2]));
    x.F[id] = (double)((T)dpe * (T)a.u_s[id]);
}

// cell divergence of F, column mass tendency and interface vertical mass
// flux (Eq. 3): one lane per column, levels from the top
template <typename T> __global__ void k_t_div(StageArgs a, TermArgs x) {
    const int i = (int)((long)blockIdx.x * blockDim.x + threadIdx.x);
    const int K = a.K;
    if (i >= a.mesh.N) return;
    const int *ce = a.mesh.c_edge + 6 * (long)i;
    const T *cd = tb<T>(a.mesh.c_div, a.mesh.c_div32) + 6 * (long)i;
    T acc = 0;
    for (int k = 0; k < K; k++) {
        T D = 0;
        for (int s = 0; s < 6; s++)
            if (ce[s] >= 0) D += cd[s] * (T)x.F[(long)ce[s] * K + k];
        acc += D;
        x.D[(long)i * K + k] = (double)acc;   // prefix sum of the divergences
    }
    const T dps = -acc;
    double *md = a.mdot + (long)i * (K + 1);
    md[0] = 0.0;
    md[K] = 0.0;
    for (int k = 0; k < K - 1; k++) md[k + 1] = (double)(-(T)x.D[(long)i * K + k] - (T)a.sig[k + 1] * dps);
    a.dps[i] = (double)dps;
}

// theta of the stage's input (FP64) and the cell kinetic energy (Eq. 5)
template <typename T> __global__ void k_t_ke(StageArgs a, TermArgs x) {
    const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int K = a.K;
    if (id >= (long)a.mesh.N * K) return;
    const int i = (int)(id / K), k = (int)(id - (long)i * K);
    x.theta[id] = a.Th_s[id] / layer_mass(a, k, a.ps_s[i]);
    const int *ce = a.mesh.c_edge + 6 * (long)i;
    const T *ck = tb<T>(a.mesh.c_ke, a.mesh.c_ke32) + 6 * (long)i;
    T kin = 0;
    for (int s = 0; s < 6; s++)
        if (ce[s] >= 0) {
            const T u = (T)a.u_s[(long)ce[s] * K + k];
            kin += ck[s] * (u * u);
        }
    ((double *)a.ke)[id] = (double)kin;
}

// quadratic-fit second derivatives of theta (the third-order flux's Hessian)
template <typename T> __global__ void k_t_hess(StageArgs a, TermArgs x) {
    const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int K = a.K;
    if (id >= (long)a.mesh.N * K) return;
    const int i = (int)(id / K), k = (int)(id - (long)i * K);
    const int *cn = a.mesh.c_nbr + 6 * (long)i;
    const T *ch = tb<T>(a.mesh.c_hess, a.mesh.c_hess32) + 18 * (long)i;
    const T th = (T)x.theta[id];
    T h0 = 0, h1 = 0, h2 = 0;
    for (int s = 0; s < 6; s++) {
        const T d = (T)x.theta[(long)cn[s] * K + k] - th;   // pad slot: the cell itself, zero weights
        h0 += ch[s] * d;
        h1 += ch[6 + s] * d;
        h2 += ch[12 + s] * d;
    }
    double *H = (double *)a.hth + (long)i * 3 * K + k;
    H[0] = (double)h0;
    H[K] = (double)h1;
    H[2 * K] = (double)h2;
}

// relative vorticity at the vertices (Eq. 5 zeta), into qv
template <typename T> __global__ void k_t_zeta(StageArgs a, TermArgs) {
    const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int K = a.K;
    if (id >= (long)a.mesh.V * K) return;
    const int v = (int)(id / K), k = (int)(id - (long)v * K);
    const T *cw = tb<T>(a.mesh.v_curl, a.mesh.v_curl32) + 4 * (long)v;
    T z = 0;
    for (int r = 0; r < 3; r++) z += cw[r] * (T)a.u_s[(long)a.mesh.v_edge[4 * (long)v + r] * K + k];
    ((double *)a.qv)[id] = (double)z;
}

// kite-weighted vertex mass and potential vorticity q = (zeta + f)/dpi_v, in place in qv
template <typename T> __global__ void k_t_pv(StageArgs a, TermArgs) {
    const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int K = a.K;
    if (id >= (long)a.mesh.V * K) return;
    const int v = (int)(id / K), k = (int)(id - (long)v * K);
    T hv = 0;
    for (int r = 0; r < 3; r++)
        hv += (T)a.mesh.v_kite[4 * (long)v + r] * (T)layer_mass(a, k, a.ps_s[a.mesh.v_cell[4 * (long)v + r]]);
    double *q = (double *)a.qv;
    q[id] = (double)(((T)q[id] + (T)a.mesh.v_f[v]) / hv);
}

// TRiSK Coriolis term (Eq. 5 zeta_p dpi u_t): each cell's half sum for each of
// its edges, with Q_s = q_v(s) + q_v(s+1) twice the PV of edge s and the
// table's weights w' = w l / (4 d):  Q_s sum_t w' F_t + sum_t w' F_t Q_t
template <typename T> __global__ void k_t_coriolis(StageArgs a, TermArgs x) {
    const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int K = a.K;
    if (id >= (long)a.mesh.N * K) return;
    const int i = (int)(id / K), k = (int)(id - (long)i * K);
    const int *ce = a.mesh.c_edge + 6 * (long)i, *cv = a.mesh.c_vert + 6 * (long)i;
    const T *cd = tb<T>(a.mesh.c_div, a.mesh.c_div32) + 6 * (long)i;
    const T *tk = tb<T>(a.mesh.c_tk, a.mesh.c_tk32) + 36 * (long)i;
    const double *qv = (const double *)a.qv;
    T F[6], QV[6], Q[6];
    for (int s = 0; s < 6; s++) {
        F[s] = ce[s] >= 0 ? (T)x.F[(long)ce[s] * K + k] : (T)0;
        QV[s] = (T)qv[(long)cv[s] * K + k];
    }
    for (int s = 0; s < 6; s++) Q[s] = QV[s] + QV[(s + 1) % 6];
    double *qh = (double *)a.qh;
    for (int s = 0; s < 6; s++) {
        if (ce[s] < 0) continue;
        T A = 0, B = 0;
        for (int t = 1; t < 6; t++) {
            const int sp = (s + t) % 6;
            A += tk[s * 6 + sp] * F[sp];
            B += tk[s * 6 + sp] * (F[sp] * Q[sp]);
        }
        const int side = cd[s] > (T)0 ? 0 : 1;
        qh[((long)ce[s] * 2 + side) * K + k] = (double)(Q[s] * A + B);
    }
}

// divergence of the third-order upwind theta flux (Eq. 4, horizontal), into D
// (the prefix sums there are no longer needed)
template <typename T> __global__ void k_t_hdiv(StageArgs a, TermArgs x) {
    const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int K = a.K;
    if (id >= (long)a.mesh.N * K) return;
    const int i = (int)(id / K), k = (int)(id - (long)i * K);
    const int *ce = a.mesh.c_edge + 6 * (long)i, *cn = a.mesh.c_nbr + 6 * (long)i;
    const T *cd = tb<T>(a.mesh.c_div, a.mesh.c_div32) + 6 * (long)i;
    const T *hd = tb<T>(a.mesh.c_hd, a.mesh.c_hd32) + 48 * (long)i;
    const double *H = (const double *)a.hth;
    const long hi0 = (long)i * 3 * K + k;
    const T Hi0 = (T)H[hi0], Hi1 = (T)H[hi0 + K], Hi2 = (T)H[hi0 + 2 * K];
    const T thi = (T)x.theta[id];
    T hdiv = 0;
    for (int s = 0; s < 6; s++) {
        if (ce[s] < 0) continue;
        const int nb = cn[s];
        const T F = (T)x.F[(long)ce[s] * K + k];
        const T *h = hd + 8 * s;
        const long hn0 = (long)nb * 3 * K + k;
        const T hi = Hi0 * h[0] + Hi1 * h[1] + Hi2 * h[2];
        const T hn = (T)H[hn0] * h[3] + (T)H[hn0 + K] * h[4] + (T)H[hn0 + 2 * K] * h[5];
        const bool up_i = (F >= (T)0) == (cd[s] > (T)0);
        const T thn = (T)x.theta[(long)nb * K + k];
        const T tv = h[6] * (up_i ? hi : hn) + (T)0.5 * (thi + thn);
        hdiv += cd[s] * (F * tv);
    }
    x.D[id] = (double)hdiv;
}

// vertical theta flux (centred, Eq. 4) and the stage update of pi_s and Theta
template <typename T> __global__ void k_t_thupd(StageArgs a, TermArgs x) {
    const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int K = a.K;
    if (id >= (long)a.mesh.N * K) return;
    const int i = (int)(id / K), k = (int)(id - (long)i * K);
    const double *md = a.mdot + (long)i * (K + 1);
    const T th = (T)x.theta[id];
    T vd = 0;
    if (k > 0) vd -= (T)md[k] * ((T)0.5 * ((T)x.theta[id - 1] + th));
    if (k < K - 1) vd += (T)md[k + 1] * ((T)0.5 * (th + (T)x.theta[id + 1]));
    const double dTh = -x.D[id] - (double)vd;
    a.Th_o[id] = a.Th_n[id] + a.dts * dTh;
    if (k == 0) a.ps_o[i] = a.ps_n[i] + a.dts * a.dps[i];
}

// column diagnostics of the updated state (Eqs. 8-9): mid-layer pressure,
// specific volume, layer geopotential integrated from phi_s; one lane per column
template <typename T> __global__ void k_t_coldiag(StageArgs a, TermArgs x) {
    const int i = (int)((long)blockIdx.x * blockDim.x + threadIdx.x);
    const int K = a.K;
    if (i >= a.mesh.N) return;
    const T ps = (T)a.ps_o[i], pt = (T)a.ptop;
    T phib = (T)a.phis[i];
    for (int k = K - 1; k >= 0; k--) {
        const long o = (long)i * K + k;
        const T dpi = (T)a.dsig[k] * (ps - pt);
        const T pk = (T)0.5 * ((pt + (T)a.sig[k] * (ps - pt)) + (pt + (T)a.sig[k + 1] * (ps - pt)));
        const T temp = ((T)a.Th_o[o] / dpi) * tpow(pk * (T)a.inv_p0, (T)a.kappa);
        const T al = (T)a.rd * temp / pk;
        const T phit = phib + al * dpi;
        a.alpha[o] = (double)al;
        a.phim[o] = (double)((T)0.5 * (phit + phib));
        x.pmid[o] = (double)pk;
        phib = phit;
    }
}

// momentum advective terms on the edge: the two cells' Coriolis shares,
// -grad K (TK) and the centred vertical advection of u (TV), summed in FP64
// into F (no longer needed)
template <typename TK, typename TV> __global__ void k_t_uadv(StageArgs a, TermArgs x) {
    const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int K = a.K;
    if (id >= (long)a.mesh.E * K) return;
    const int e = (int)(id / K), k = (int)(id - (long)e * K);
    const int c1 = a.mesh.e_cell[2 * e], c2 = a.mesh.e_cell[2 * e + 1];
    const double *qh = (const double *)a.qh, *ke = (const double *)a.ke;
    const double cor = qh[((long)e * 2) * K + k] + qh[((long)e * 2 + 1) * K + k];
    const TK gk = -((TK)ke[(long)c2 * K + k] - (TK)ke[(long)c1 * K + k]) * tb<TK>(a.mesh.e_dinv, a.mesh.e_dinv32)[e];
    const long K1 = K + 1;
    const TV mt = (TV)0.5 * ((TV)a.mdot[(long)c1 * K1 + k] + (TV)a.mdot[(long)c2 * K1 + k]);
    const TV mb = (TV)0.5 * ((TV)a.mdot[(long)c1 * K1 + k + 1] + (TV)a.mdot[(long)c2 * K1 + k + 1]);
    const TV uk = (TV)a.u_s[id];
    TV va = 0;
    if (k < K - 1) va += mb * ((TV)a.u_s[id + 1] - uk);
    if (k > 0) va += mt * (uk - (TV)a.u_s[id - 1]);
    const double dpe = 0.5 * (layer_mass(a, k, a.ps_s[c1]) + layer_mass(a, k, a.ps_s[c2]));
    va = va / (TV)(2.0 * dpe);
    x.F[id] = cor + (double)gk - (double)va;
}

// pressure-gradient force and gravity (Eq. 5) from the updated state's
// column diagnostics, and the stage update of u
template <typename T> __global__ void k_t_pgf(StageArgs a, TermArgs x) {
    const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int K = a.K;
    if (id >= (long)a.mesh.E * K) return;
    const int e = (int)(id / K), k = (int)(id - (long)e * K);
    const long x1 = (long)a.mesh.e_cell[2 * e] * K + k, x2 = (long)a.mesh.e_cell[2 * e + 1] * K + k;
    const T ae = (T)0.5 * ((T)a.alpha[x1] + (T)a.alpha[x2]);
    const T pg = -(ae * ((T)x.pmid[x2] - (T)x.pmid[x1]) + ((T)a.phim[x2] - (T)a.phim[x1])) *
                 tb<T>(a.mesh.e_dinv, a.mesh.e_dinv32)[e];
    a.u_o[id] = a.u_n[id] + a.dts * (x.F[id] + (double)pg);
}

#define MPDC_TERM_LAUNCH(kernel, bit, n)                                                              \
    do {                                                                                           \
        if (x.mask & (1u << (bit)))                                                                \
            hipLaunchKernelGGL(kernel<float>, dim3(tgrid(n)), dim3(256), 0, s, a, x);              \
        else                                                                                       \
            hipLaunchKernelGGL(kernel<double>, dim3(tgrid(n)), dim3(256), 0, s, a, x);             \
    } while (0)

}  // namespace

hipError_t launch_term_stage(const StageArgs &a, const TermArgs &x, hipStream_t s) {
    const long N = a.mesh.N, E = a.mesh.E, V = a.mesh.V, K = a.K;
    MPDC_TERM_LAUNCH(k_t_flux, TERM_MASS_FLUX, E * K);
    MPDC_TERM_LAUNCH(k_t_div, TERM_DIVERGENCE, N);
    MPDC_TERM_LAUNCH(k_t_ke, TERM_KINETIC_ENERGY, N * K);
    MPDC_TERM_LAUNCH(k_t_hess, TERM_THETA_FLUX, N * K);
    MPDC_TERM_LAUNCH(k_t_zeta, TERM_VORTICITY, V * K);
    MPDC_TERM_LAUNCH(k_t_pv, TERM_VERTEX_MASS, V * K);
    MPDC_TERM_LAUNCH(k_t_coriolis, TERM_CORIOLIS, N * K);
    MPDC_TERM_LAUNCH(k_t_hdiv, TERM_THETA_FLUX, N * K);
    MPDC_TERM_LAUNCH(k_t_thupd, TERM_VERTICAL_ADVECTION, N * K);
    MPDC_TERM_LAUNCH(k_t_coldiag, TERM_COLUMN_DIAG, N);
    {
        const bool fk = x.mask & (1u << TERM_KINETIC_ENERGY), fv = x.mask & (1u << TERM_VERTICAL_ADVECTION);
        const dim3 g(tgrid(E * K)), b(256);
        if (fk && fv) hipLaunchKernelGGL((k_t_uadv<float, float>), g, b, 0, s, a, x);
        else if (fk) hipLaunchKernelGGL((k_t_uadv<float, double>), g, b, 0, s, a, x);
        else if (fv) hipLaunchKernelGGL((k_t_uadv<double, float>), g, b, 0, s, a, x);
        else hipLaunchKernelGGL((k_t_uadv<double, double>), g, b, 0, s, a, x);
    }
    MPDC_TERM_LAUNCH(k_t_pgf, TERM_PRESSURE_GRADIENT, E * K);
    return hipGetLastError();
}

}  // namespace mpdc
