// HIP kernels of the dry dynamical core for gfx950 (MI355X).
//
// One RK3 stage of the shallow-water (SW), hydrostatic (HDC) and
// non-hydrostatic (NDC) C-grid dycore, written for a level- and
// member-innermost layout ([entity][k][m]): consecutive lanes of a wavefront
// handle consecutive (k, m) of one entity, so every stencil gather reads a
// contiguous run of K*M values and every store is coalesced.
//
// Per stage (tendencies from the previous stage y^(s-1), base state y^n):
//   cell_a  (cell columns)  divergence of the mass flux, column mass tendency
//                           and vertical mass flux (Eq. 3, LDS prefix sum),
//                           kinetic energy, second derivatives of theta;
//                           NDC: explicit advective step of w and phi (Eqs. 6-7)
//   vertex  (vertex x km)   vorticity, FP64 vertex mass, potential vorticity
//   cell_b  (cell columns)  theta_m flux-form transport (Eq. 4, third-order
//                           upwind) and the mass/Theta update; then the FP64
//                           column diagnostics of the updated state: pressure,
//                           alpha and the hydrostatic geopotential (Eq. 8, LDS
//                           scan), or for NDC the equation of state (Eq. 9) and
//                           the implicit vertical acoustic solve (HEVI)
//   edge    (edge x km)     TRiSK Coriolis term, kinetic-energy gradient,
//                           vertical advection of u, FP64 pressure-gradient and
//                           gravity term (Eq. 5), RK update of u
// The mass flux F = dpi_e u is recomputed by each consumer from u and the
// 2-D surface pressure instead of being stored: that reads as many bytes as
// a stored F would and saves writing it.
//
// Template parameter R is the arithmetic type of the advective terms:
// double for the all-FP64 policy, float for the mixed policy.  Everything
// the mixed policy keeps in FP64 (mass sums, vertex mass and the PV
// division, pressure gradient, gravity/geopotential, the column solve, the
// state update) is double in both instantiations.
#include <hip/hip_runtime.h>

#include "dycore_kernels.h"

namespace mpdc {

template <typename R> __device__ __forceinline__ const R *pick(const double *d, const float *f);
template <> __device__ __forceinline__ const double *pick<double>(const double *d, const float *) { return d; }
template <> __device__ __forceinline__ const float *pick<float>(const double *, const float *f) { return f; }

// layer mass of layer k for surface pressure ps (HDC/NDC) or depth h (SW)
template <int MODEL>
__device__ __forceinline__ double layer_mass(const StageArgs &a, int k, double ps) {
    if (MODEL == MODEL_SW) return ps;
    return a.dsig[k] * (ps - a.ptop);
}

// u of the previous stage in the advective precision
template <typename R>
__device__ __forceinline__ R u_prev(const StageArgs &a, long idx) {
    if constexpr (sizeof(R) == 8) return a.u_s[idx];
    else return a.u32_s[idx];
}

// theta of the previous stage in the advective precision
template <int MODEL, typename R>
__device__ __forceinline__ R theta_prev(const StageArgs &a, int i, int k, int mm) {
    const long KM = (long)a.K * a.M;
    const long idx = (long)i * KM + (long)k * a.M + mm;
    if constexpr (sizeof(R) == 8) {
        double dpi = layer_mass<MODEL>(a, k, a.ps_s[(long)i * a.M + mm]);
        return a.Th_s[idx] / dpi;
    } else {
        return a.th32_s[idx];
    }
}

// ---------------------------------------------------------------------------
// cell_a
// ---------------------------------------------------------------------------
template <int MODEL, typename R>
__global__ void __launch_bounds__(1024) k_cell_a(StageArgs a) {
    extern __shared__ double lds[];
    const DevMesh &m = a.mesh;
    const int K = a.K, M = a.M, KM = K * M;
    const int tid = threadIdx.x;
    const int lc = tid / KM;
    const int km = tid - lc * KM;
    const int i = blockIdx.x * a.cpb + lc;
    const bool valid = (lc < a.cpb) && (i < m.N);
    const int k = km / M, mm = km - k * M;
    double *sD = lds;                           // [cpb][KM]
    double *sMd = lds + a.cpb * KM;             // [cpb][(K+1) M]  (NDC)

    double D = 0.0;
    double ps_i = 0.0;
    R ke = 0;
    if (valid) {
        ps_i = a.ps_s[(long)i * M + mm];
        const double dpi_i = layer_mass<MODEL>(a, k, ps_i);
        const double *cdiv = m.c_div + (long)i * kCellSlots;
        const R *cke = pick<R>(m.c_ke, m.c_ke32) + (long)i * kCellSlots;
#pragma unroll
        for (int j = 0; j < kCellSlots; j++) {
            const int e = m.c_edge[(long)i * kCellSlots + j];
            if (e < 0) continue;
            const int nb = m.c_nbr[(long)i * kCellSlots + j];
            const double dpi_nb = layer_mass<MODEL>(a, k, a.ps_s[(long)nb * M + mm]);
            const double dpe = 0.5 * (dpi_i + dpi_nb);
            const R ue = u_prev<R>(a, (long)e * KM + km);
            if constexpr (sizeof(R) == 8) {
                D += cdiv[j] * (dpe * ue);
            } else {
                const float F32 = (float)dpe * ue;
                D += cdiv[j] * (double)F32;
            }
            ke += cke[j] * ue * ue;
        }
        a.ke_out<R>()[(long)i * KM + km] = ke;
    }

    if constexpr (MODEL == MODEL_SW) {
        if (valid) {
            // h^(s) = h^n - dt_s D  (forward part of the stage)
            const long x = (long)i * M + mm;
            const double hn = a.ps_n[x];
            a.ps_o[x] = hn + a.dts * (-D);
        }
        return;
    } else {
        // ---- column mass tendency and vertical mass flux (LDS scan) ----
        if (valid) sD[lc * KM + km] = D;
        __syncthreads();
        double dps = 0.0, mdot_b = 0.0;
        if (valid) {
            double s = 0.0;
            for (int j = 0; j < K; j++) s += sD[lc * KM + j * M + mm];
            dps = -s;
            double acc = 0.0;
            for (int j = 0; j <= k; j++) acc += sD[lc * KM + j * M + mm];
            mdot_b = (k == K - 1) ? 0.0 : -acc - a.sig[k + 1] * dps;
            const long K1M = (long)(K + 1) * M;
            a.mdot[(long)i * K1M + (long)(k + 1) * M + mm] = mdot_b;
            if (k == 0) {
                a.mdot[(long)i * K1M + mm] = 0.0;
                a.dps[(long)i * M + mm] = dps;
            }
        }

        // ---- second derivatives of theta (quadratic fit) ----
        if (valid) {
            const R th_i = theta_prev<MODEL, R>(a, i, k, mm);
            const R *ch = pick<R>(m.c_hess, m.c_hess32) + (long)i * 3 * kCellSlots;
            R h0 = 0, h1 = 0, h2 = 0;
#pragma unroll
            for (int j = 0; j < kCellSlots; j++) {
                const int nb = m.c_nbr[(long)i * kCellSlots + j];
                const R dth = theta_prev<MODEL, R>(a, nb, k, mm) - th_i;
                h0 += ch[j] * dth;
                h1 += ch[kCellSlots + j] * dth;
                h2 += ch[2 * kCellSlots + j] * dth;
            }
            R *H = a.hth_out<R>() + (long)i * 3 * KM;
            H[km] = h0;
            H[KM + km] = h1;
            H[2 * KM + km] = h2;
        }

        if constexpr (MODEL == MODEL_NDC) {
            // ---- explicit advective step of w and phi at interface k ----
            const int K1 = K + 1;
            if (valid) {
                sMd[lc * K1 * M + (k + 1) * M + mm] = mdot_b;
                if (k == 0) sMd[lc * K1 * M + mm] = 0.0;
            }
            __syncthreads();
            if (valid) {
                const long K1M = (long)K1 * M;
                const double *md = sMd + lc * K1 * M;
                const double *wn = a.w_n + (long)i * K1M;
                const double *pn = a.phi_n + (long)i * K1M;
                const double *ws = a.w_s + (long)i * K1M;
                const double *phs = a.phi_s + (long)i * K1M;
                // interface masses from the previous stage's layer masses
                const double dk = layer_mass<MODEL>(a, k, ps_i);
                const double dkm = (k > 0) ? layer_mass<MODEL>(a, k - 1, ps_i) : 0.0;
                const double dh = (k == 0) ? 0.5 * dk : 0.5 * (dkm + dk);
                const double *cdiv = m.c_div + (long)i * kCellSlots;
                R aw = 0, ap = 0;
                const double wi = ws[(long)k * M + mm], pi_ = phs[(long)k * M + mm];
#pragma unroll
                for (int j = 0; j < kCellSlots; j++) {
                    const int e = m.c_edge[(long)i * kCellSlots + j];
                    if (e < 0) continue;
                    const int nb = m.c_nbr[(long)i * kCellSlots + j];
                    const double psnb = a.ps_s[(long)nb * M + mm];
                    // mass flux averaged to interface k (half of layer 0 at the top)
                    const double dpe_k = 0.5 * (dk + layer_mass<MODEL>(a, k, psnb));
                    const double Fk = dpe_k * (double)u_prev<R>(a, (long)e * KM + km);
                    double Fh;
                    if (k == 0) {
                        Fh = 0.5 * Fk;
                    } else {
                        const double dpe_m = 0.5 * (dkm + layer_mass<MODEL>(a, k - 1, psnb));
                        const double Fm = dpe_m * (double)u_prev<R>(a, (long)e * KM + km - M);
                        Fh = 0.5 * (Fm + Fk);
                    }
                    const long nbo = (long)nb * K1M + (long)k * M + mm;
                    if constexpr (sizeof(R) == 8) {
                        aw += cdiv[j] * Fh * 0.5 * (a.w_s[nbo] - wi);
                        ap += cdiv[j] * Fh * 0.5 * (a.phi_s[nbo] - pi_);
                    } else {
                        const float c = (float)cdiv[j] * (float)Fh * 0.5f;
                        aw += c * (float)(a.w_s[nbo] - wi);
                        ap += c * (float)(a.phi_s[nbo] - pi_);
                    }
                }
                const R inv_dh = (R)(1.0 / dh);
                R vw = 0, vp = 0;
                if (k >= 1) {
                    const R ml = (R)(0.5 * (md[(k - 1) * M + mm] + md[k * M + mm]));
                    vw += ml * (R)(wi - ws[(long)(k - 1) * M + mm]);
                    vp += ml * (R)(pi_ - phs[(long)(k - 1) * M + mm]);
                }
                {
                    const R ml = (R)(0.5 * (md[k * M + mm] + md[(k + 1) * M + mm]));
                    vw += ml * (R)(ws[(long)(k + 1) * M + mm] - wi);
                    vp += ml * (R)(phs[(long)(k + 1) * M + mm] - pi_);
                }
                const R advw = aw * inv_dh + vw * (inv_dh * (R)0.5);
                const R advp = ap * inv_dh + vp * (inv_dh * (R)0.5);
                const long o = (long)i * K1M + (long)k * M + mm;
                a.wstar[o] = (k == 0) ? 0.0 : wn[(long)k * M + mm] - a.dts * (double)advw;
                a.phistar[o] = pn[(long)k * M + mm] - a.dts * (double)advp;
                if (k == K - 1) {
                    a.wstar[o + M] = 0.0;
                    a.phistar[o + M] = pn[(long)K * M + mm];
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// vertex: vorticity, FP64 vertex mass, potential vorticity
// ---------------------------------------------------------------------------
template <int MODEL, typename R>
__global__ void __launch_bounds__(1024) k_vertex(StageArgs a) {
    const DevMesh &m = a.mesh;
    const int KM = a.K * a.M;
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)m.V * KM) return;
    const int v = (int)(idx / KM);
    const int km = (int)(idx - (long)v * KM);
    const int k = km / a.M, mm = km - k * a.M;
    const R *cw = pick<R>(m.v_curl, m.v_curl32) + (long)v * 3;
    R zeta = 0;
    double hv = 0.0;
#pragma unroll
    for (int j = 0; j < 3; j++) {
        const int e = m.v_edge[(long)v * 3 + j];
        zeta += cw[j] * u_prev<R>(a, (long)e * KM + km);
        const int c = m.v_cell[(long)v * 3 + j];
        hv += m.v_kite[(long)v * 3 + j] * layer_mass<MODEL>(a, k, a.ps_s[(long)c * a.M + mm]);
    }
    a.qv_out<R>()[idx] = (R)(((double)zeta + m.v_f[v]) / hv);
}

// ---------------------------------------------------------------------------
// cell_b: theta transport, mass/Theta update, column diagnostics / NH solve
// ---------------------------------------------------------------------------
template <int MODEL, typename R>
__global__ void __launch_bounds__(1024) k_cell_b(StageArgs a) {
    extern __shared__ double lds[];
    const DevMesh &m = a.mesh;
    const int K = a.K, M = a.M, KM = K * M;
    const int tid = threadIdx.x;
    const int lc = tid / KM;
    const int km = tid - lc * KM;
    const int i = blockIdx.x * a.cpb + lc;
    const bool valid = (lc < a.cpb) && (i < m.N);
    const int k = km / M, mm = km - k * M;

    double Th_new = 0.0, ps_new = 0.0;
    if (valid) {
        const double ps_i = a.ps_s[(long)i * M + mm];
        const double dpi_i = layer_mass<MODEL>(a, k, ps_i);
        const R th_i = theta_prev<MODEL, R>(a, i, k, mm);
        const R *Hs = a.hth_in<R>();
        const R Hi0 = Hs[(long)i * 3 * KM + km], Hi1 = Hs[(long)i * 3 * KM + KM + km],
                Hi2 = Hs[(long)i * 3 * KM + 2 * KM + km];
        const R *cdiv = pick<R>(m.c_div, m.c_div32) + (long)i * kCellSlots;
        const R *hdir = pick<R>(m.e_hdir, m.e_hdir32);
        const R *d2 = pick<R>(m.e_d2, m.e_d2_32);
        R hdiv = 0;
#pragma unroll
        for (int j = 0; j < kCellSlots; j++) {
            const int e = m.c_edge[(long)i * kCellSlots + j];
            if (e < 0) continue;
            const int nb = m.c_nbr[(long)i * kCellSlots + j];
            const int side = (m.e_cell[2 * (long)e] == i) ? 0 : 1;
            const double dpe = 0.5 * (dpi_i + layer_mass<MODEL>(a, k, a.ps_s[(long)nb * M + mm]));
            const R ue = u_prev<R>(a, (long)e * KM + km);
            R F;
            if constexpr (sizeof(R) == 8) F = dpe * ue;
            else F = (float)dpe * ue;
            const R th_nb = theta_prev<MODEL, R>(a, nb, k, mm);
            const long hb = (long)nb * 3 * KM + km;
            const R *ds = hdir + (long)e * 6 + side * 3;        // direction in i's frame
            const R *dn = hdir + (long)e * 6 + (1 - side) * 3;  // direction in nb's frame
            const R qi = Hi0 * ds[0] + Hi1 * ds[1] + Hi2 * ds[2];
            const R qn = Hs[hb] * dn[0] + Hs[hb + KM] * dn[1] + Hs[hb + 2 * KM] * dn[2];
            // edge value with c1/c2 ordering of the edge
            const R q1 = side ? th_nb : th_i, q2 = side ? th_i : th_nb;
            const R h1 = side ? qn : qi, h2 = side ? qi : qn;
            const R c = d2[e];
            const R sg = (F >= (R)0) ? (R)1 : (R)-1;
            const R tv = (R)0.5 * (q1 + q2) - c * (h1 + h2) + sg * c * (h2 - h1);
            hdiv += cdiv[j] * (F * tv);
        }
        // vertical theta flux through the layer's interfaces (centred theta)
        const long K1M = (long)(K + 1) * M;
        const double *md = a.mdot + (long)i * K1M;
        R top = 0, bot = 0;
        if (k > 0) top = (R)md[(long)k * M + mm] * ((R)0.5 * (theta_prev<MODEL, R>(a, i, k - 1, mm) + th_i));
        if (k < K - 1) bot = (R)md[(long)(k + 1) * M + mm] * ((R)0.5 * (th_i + theta_prev<MODEL, R>(a, i, k + 1, mm)));
        const R dTh = -hdiv - (bot - top);
        const long x = (long)i * KM + km;
        Th_new = a.Th_n[x] + a.dts * (double)dTh;
        ps_new = a.ps_n[(long)i * M + mm] + a.dts * a.dps[(long)i * M + mm];
        (void)dpi_i;
    }
    // all reads of ps_n / Th_n happen before this barrier (stage 3 writes in place)
    double *sA = lds;                       // [cpb][KM]
    __syncthreads();

    if constexpr (MODEL == MODEL_HDC) {
        double pk = 0.0, al = 0.0, dpn = 0.0;
        if (valid) {
            const long x = (long)i * KM + km;
            a.Th_o[x] = Th_new;
            if (k == 0) a.ps_o[(long)i * M + mm] = ps_new;
            const double pit = a.ptop + a.sig[k] * (ps_new - a.ptop);
            const double pib = a.ptop + a.sig[k + 1] * (ps_new - a.ptop);
            dpn = a.dsig[k] * (ps_new - a.ptop);
            pk = 0.5 * (pit + pib);
            const double th = Th_new / dpn;
            const double T = th * pow(pk / a.p0, a.kappa);
            al = a.rd * T / pk;
            sA[lc * KM + km] = al * dpn;
            if (a.th32_o) a.th32_o[x] = (float)th;
        }
        __syncthreads();
        if (valid) {
            // hydrostatic geopotential from the flat surface upwards (Eq. 8)
            double acc = 0.0;
            for (int j = K - 1; j > k; j--) acc += sA[lc * KM + j * M + mm];
            const double phit = acc + sA[lc * KM + k * M + mm];
            const long x = (long)i * KM + km;
            a.alpha[x] = al;
            a.phim[x] = 0.5 * (phit + acc);
        }
    } else if constexpr (MODEL == MODEL_NDC) {
        // ---- implicit vertical acoustic solve of the column (FP64) ----
        const int K1 = K + 1;
        const long K1M = (long)K1 * M;
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
        double dpn = 0.0, phs_k = 0.0, phs_k1 = 0.0, ws_k = 0.0;
        if (valid) {
            const long x = (long)i * KM + km;
            a.Th_o[x] = Th_new;
            if (k == 0) a.ps_o[(long)i * M + mm] = ps_new;
            dpn = a.dsig[k] * (ps_new - a.ptop);
            phs_k = a.phistar[(long)i * K1M + (long)k * M + mm];
            phs_k1 = a.phistar[(long)i * K1M + (long)(k + 1) * M + mm];
            ws_k = a.wstar[(long)i * K1M + (long)k * M + mm];
            const double dphi = phs_k - phs_k1;
            const double p = a.p0 * pow(a.rd * Th_new / (a.p0 * dphi), a.gamma);
            sP[base + km] = p;
            sC[base + km] = a.gamma * a.grav * a.dts * p / dphi;
        }
        __syncthreads();
        if (valid && k >= 1) {
            // row r = k-1 for interior interface k (between layers k-1 and k)
            const double dpm = a.dsig[k - 1] * (ps_new - a.ptop);
            const double D = a.grav * a.dts / (0.5 * (dpm + dpn));
            const double Cm = sC[base + (k - 1) * M + mm], Ck = sC[base + km];
            const int r = (k - 1) * M + mm;
            sSub[base + r] = -D * Cm;
            sDia[base + r] = 1.0 + D * (Cm + Ck);
            sSup[base + r] = -D * Ck;
            sRhs[base + r] = ws_k + D * (sP[base + km] - sP[base + (k - 1) * M + mm]) - a.grav * a.dts;
        }
        __syncthreads();
        if (valid && k == 0) {
            // Thomas algorithm over the K-1 interior interfaces of member mm
            const int n = K - 1;
            if (n > 0) {
                double den = sDia[base + mm];
                sCp[base + mm] = sSup[base + mm] / den;
                sDp[base + mm] = sRhs[base + mm] / den;
                for (int r = 1; r < n; r++) {
                    const int o = base + r * M + mm, op = base + (r - 1) * M + mm;
                    den = sDia[o] - sSub[o] * sCp[op];
                    sCp[o] = (r < n - 1) ? sSup[o] / den : 0.0;
                    sDp[o] = (sRhs[o] - sSub[o] * sDp[op]) / den;
                }
                // back substitution: the solution overwrites sDp
                for (int r = n - 2; r >= 0; r--) {
                    const int o = base + r * M + mm;
                    sDp[o] = sDp[o] - sCp[o] * sDp[o + M];
                }
            }
        }
        __syncthreads();
        double wk = 0.0, phk = 0.0;
        if (valid) {
            wk = (k == 0) ? 0.0 : sDp[base + (k - 1) * M + mm];
            phk = phs_k + a.grav * a.dts * wk;
            sPhi[lc * K1 * M + k * M + mm] = phk;
            if (k == K - 1) sPhi[lc * K1 * M + K * M + mm] = phs_k1;   // surface: w = 0
            const long o = (long)i * K1M + (long)k * M + mm;
            a.w_o[o] = wk;
            a.phi_o[o] = phk;
            if (k == K - 1) {
                a.w_o[o + M] = 0.0;
                a.phi_o[o + M] = phs_k1;
            }
        }
        __syncthreads();
        double pk = 0.0, dphi = 0.0;
        if (valid) {
            const double phb = sPhi[lc * K1 * M + (k + 1) * M + mm];
            dphi = phk - phb;
            pk = a.p0 * pow(a.rd * Th_new / (a.p0 * dphi), a.gamma);
            sPn[base + km] = pk;
            const long x = (long)i * KM + km;
            a.alpha[x] = dphi / dpn;
            a.pm[x] = pk;
            a.phim[x] = 0.5 * (phk + phb);
            if (a.th32_o) a.th32_o[x] = (float)(Th_new / dpn);
        }
        __syncthreads();
        if (valid) {
            // mu = dp/dpi at interfaces, copied to the ends, averaged to the layer
            auto mu_at = [&](int kk) -> double {
                if (K == 1) return 1.0;
                if (kk < 1) kk = 1;
                if (kk > K - 1) kk = K - 1;
                const double dp_a = a.dsig[kk - 1] * (ps_new - a.ptop);
                const double dp_b = a.dsig[kk] * (ps_new - a.ptop);
                return (sPn[base + kk * M + mm] - sPn[base + (kk - 1) * M + mm]) / (0.5 * (dp_a + dp_b));
            };
            a.mum[(long)i * KM + km] = 0.5 * (mu_at(k) + mu_at(k + 1));
        }
    }
}

// ---------------------------------------------------------------------------
// edge: momentum
// ---------------------------------------------------------------------------
// Each lane owns L consecutive (k, m) values of one edge, so every gather is
// one L-wide vector load and the per-edge table lookups are shared by L
// values.  With M == 1 the L values are consecutive levels; with M > 1 they
// are consecutive members of one level (L divides M).
template <typename T, int L> struct alignas(sizeof(T) * L) Pack {
    T v[L];
};
template <typename T, int L> __device__ __forceinline__ Pack<T, L> ldp(const T *p) {
    return *reinterpret_cast<const Pack<T, L> *>(p);
}
template <typename T, int L> __device__ __forceinline__ void stp(T *p, const Pack<T, L> &x) {
    *reinterpret_cast<Pack<T, L> *>(p) = x;
}

template <int MODEL, typename R, int L, bool M1>
__global__ void __launch_bounds__(1024) k_edge(StageArgs a) {
    const DevMesh &m = a.mesh;
    const int K = a.K, M = M1 ? 1 : a.M, KM = K * M;
    const int lanes = KM / L;                       // lanes per edge
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)m.E * lanes) return;
    const int e = (int)(idx / lanes);
    const int km0 = (int)(idx - (long)e * lanes) * L;
    const long base = (long)e * KM + km0;
    constexpr bool m1 = M1;
    const int k0 = M1 ? km0 : km0 / M, mm0 = km0 - k0 * M;   // M > 1: all L values share level k0
    int kk[L];
    double dsg[L];                                   // layer sigma thickness of each value
#pragma unroll
    for (int j = 0; j < L; j++) {
        kk[j] = m1 ? k0 + j : k0;
        dsg[j] = (MODEL == MODEL_SW) ? 1.0 : a.dsig[kk[j]];
    }

    // layer mass of the L values at cell c of the previous stage
    auto dpi_at = [&](int c, double out[L]) {
        if (m1) {
            const double s = a.ps_s[c];
#pragma unroll
            for (int j = 0; j < L; j++) out[j] = (MODEL == MODEL_SW) ? s : dsg[j] * (s - a.ptop);
        } else {
            const Pack<double, L> s = ldp<double, L>(a.ps_s + (long)c * M + mm0);
#pragma unroll
            for (int j = 0; j < L; j++) out[j] = (MODEL == MODEL_SW) ? s.v[j] : dsg[j] * (s.v[j] - a.ptop);
        }
    };

    const int c1 = m.e_cell[2 * (long)e], c2 = m.e_cell[2 * (long)e + 1];
    const int v1 = m.e_vert[2 * (long)e], v2 = m.e_vert[2 * (long)e + 1];
    const R *qv = a.qv_in<R>();
    const R *ke = a.ke_in<R>();

    // TRiSK Coriolis term: sum_e' w l_e'/d_e F_e' (q_e + q_e')/2
    R qe[L], Q[L];
    {
        const Pack<R, L> qa = ldp<R, L>(qv + (long)v1 * KM + km0), qb = ldp<R, L>(qv + (long)v2 * KM + km0);
#pragma unroll
        for (int j = 0; j < L; j++) {
            qe[j] = (R)0.5 * (qa.v[j] + qb.v[j]);
            Q[j] = 0;
        }
    }
    const R *tkw = pick<R>(m.e_tkw, m.e_tkw32) + (long)e * kTriskSlots;
#pragma unroll
    for (int t = 0; t < kTriskSlots; t++) {
        const int ep = m.e_tk[(long)e * kTriskSlots + t];
        if (ep < 0) continue;
        const int a1 = m.e_cell[2 * (long)ep], a2 = m.e_cell[2 * (long)ep + 1];
        const int w1 = m.e_vert[2 * (long)ep], w2 = m.e_vert[2 * (long)ep + 1];
        double d1[L], d2[L];
        dpi_at(a1, d1);
        dpi_at(a2, d2);
        const Pack<R, L> up = ldp<R, L>((sizeof(R) == 8 ? (const R *)a.u_s : (const R *)a.u32_s) + (long)ep * KM + km0);
        const Pack<R, L> qa = ldp<R, L>(qv + (long)w1 * KM + km0), qb = ldp<R, L>(qv + (long)w2 * KM + km0);
        const R wt = tkw[t];
#pragma unroll
        for (int j = 0; j < L; j++) {
            const double dpe = 0.5 * (d1[j] + d2[j]);
            R F;
            if constexpr (sizeof(R) == 8) F = dpe * up.v[j];
            else F = (float)dpe * up.v[j];
            const R qep = (R)0.5 * (qa.v[j] + qb.v[j]);
            Q[j] += wt * F * ((R)0.5 * (qe[j] + qep));
        }
    }
    const R dinv = pick<R>(m.e_dinv, m.e_dinv32)[e];
    R adv[L];
    {
        const Pack<R, L> k1 = ldp<R, L>(ke + (long)c1 * KM + km0), k2 = ldp<R, L>(ke + (long)c2 * KM + km0);
#pragma unroll
        for (int j = 0; j < L; j++) adv[j] = Q[j] - (k2.v[j] - k1.v[j]) * dinv;
    }

    if constexpr (MODEL != MODEL_SW) {
        // centred vertical advection of u by the interface mass flux
        const R *us = (sizeof(R) == 8) ? (const R *)a.u_s : (const R *)a.u32_s;
        const long K1M = (long)(K + 1) * M;
        double e1[L], e2[L];
        dpi_at(c1, e1);
        dpi_at(c2, e2);
        const Pack<R, L> uk = ldp<R, L>(us + base);
        // u one level above / below each value, and the interface mass fluxes
        // at the top (k) and bottom (k+1) of each value's layer
        R uup[L], udn[L];
        double mt[L], mb[L];
        if (m1) {
#pragma unroll
            for (int j = 0; j < L; j++) {
                uup[j] = (j > 0) ? uk.v[j - 1] : ((k0 > 0) ? us[base - 1] : (R)0);
                udn[j] = (j < L - 1) ? uk.v[j + 1] : ((kk[j] < K - 1) ? us[base + L] : (R)0);
            }
            const double *m1p = a.mdot + (long)c1 * K1M + k0, *m2p = a.mdot + (long)c2 * K1M + k0;
            double i1[L + 1], i2[L + 1];
#pragma unroll
            for (int j = 0; j <= L; j++) {
                i1[j] = m1p[j];
                i2[j] = m2p[j];
            }
#pragma unroll
            for (int j = 0; j < L; j++) {
                mt[j] = 0.5 * (i1[j] + i2[j]);
                mb[j] = 0.5 * (i1[j + 1] + i2[j + 1]);
            }
        } else {
            Pack<R, L> pu, pd;
            if (k0 > 0) pu = ldp<R, L>(us + base - M);
            if (k0 < K - 1) pd = ldp<R, L>(us + base + M);
            const Pack<double, L> t1 = ldp<double, L>(a.mdot + (long)c1 * K1M + (long)k0 * M + mm0);
            const Pack<double, L> t2 = ldp<double, L>(a.mdot + (long)c2 * K1M + (long)k0 * M + mm0);
            const Pack<double, L> b1 = ldp<double, L>(a.mdot + (long)c1 * K1M + (long)(k0 + 1) * M + mm0);
            const Pack<double, L> b2 = ldp<double, L>(a.mdot + (long)c2 * K1M + (long)(k0 + 1) * M + mm0);
#pragma unroll
            for (int j = 0; j < L; j++) {
                uup[j] = (k0 > 0) ? pu.v[j] : (R)0;
                udn[j] = (k0 < K - 1) ? pd.v[j] : (R)0;
                mt[j] = 0.5 * (t1.v[j] + t2.v[j]);
                mb[j] = 0.5 * (b1.v[j] + b2.v[j]);
            }
        }
#pragma unroll
        for (int j = 0; j < L; j++) {
            const double dpe = 0.5 * (e1[j] + e2[j]);
            R va = 0;
            if (kk[j] < K - 1) va += (R)mb[j] * (udn[j] - uk.v[j]);
            if (kk[j] > 0) va += (R)mt[j] * (uk.v[j] - uup[j]);
            va = va / (R)(2.0 * dpe);
            adv[j] = adv[j] - va;
        }
    }

    // pressure-gradient force and gravity in FP64 from the updated mass/Theta
    const double dinv64 = m.e_dinv[e];
    double pgf[L];
    if constexpr (MODEL == MODEL_SW) {
        const Pack<double, L> h1 = ldp<double, L>(a.ps_o + (long)c1 * M + mm0);
        const Pack<double, L> h2 = ldp<double, L>(a.ps_o + (long)c2 * M + mm0);
#pragma unroll
        for (int j = 0; j < L; j++) pgf[j] = -a.grav * ((h2.v[j] + a.b[c2]) - (h1.v[j] + a.b[c1])) * dinv64;
    } else {
        const long x1 = (long)c1 * KM + km0, x2 = (long)c2 * KM + km0;
        const Pack<double, L> al1 = ldp<double, L>(a.alpha + x1), al2 = ldp<double, L>(a.alpha + x2);
        const Pack<double, L> ph1 = ldp<double, L>(a.phim + x1), ph2 = ldp<double, L>(a.phim + x2);
        if constexpr (MODEL == MODEL_HDC) {
            double s1[L], s2[L];
            if (m1) {
#pragma unroll
                for (int j = 0; j < L; j++) {
                    s1[j] = a.ps_o[c1];
                    s2[j] = a.ps_o[c2];
                }
            } else {
                const Pack<double, L> q1 = ldp<double, L>(a.ps_o + (long)c1 * M + mm0);
                const Pack<double, L> q2 = ldp<double, L>(a.ps_o + (long)c2 * M + mm0);
#pragma unroll
                for (int j = 0; j < L; j++) {
                    s1[j] = q1.v[j];
                    s2[j] = q2.v[j];
                }
            }
#pragma unroll
            for (int j = 0; j < L; j++) {
                const int k = kk[j];
                const double p1 = 0.5 * ((a.ptop + a.sig[k] * (s1[j] - a.ptop)) + (a.ptop + a.sig[k + 1] * (s1[j] - a.ptop)));
                const double p2 = 0.5 * ((a.ptop + a.sig[k] * (s2[j] - a.ptop)) + (a.ptop + a.sig[k + 1] * (s2[j] - a.ptop)));
                const double ae = 0.5 * (al1.v[j] + al2.v[j]);
                pgf[j] = -(ae * (p2 - p1) + (ph2.v[j] - ph1.v[j])) * dinv64;
            }
        } else {
            const Pack<double, L> p1 = ldp<double, L>(a.pm + x1), p2 = ldp<double, L>(a.pm + x2);
            const Pack<double, L> u1 = ldp<double, L>(a.mum + x1), u2 = ldp<double, L>(a.mum + x2);
#pragma unroll
            for (int j = 0; j < L; j++) {
                const double ae = 0.5 * (al1.v[j] + al2.v[j]);
                const double me = 0.5 * (u1.v[j] + u2.v[j]);
                pgf[j] = -(ae * (p2.v[j] - p1.v[j]) + me * (ph2.v[j] - ph1.v[j])) * dinv64;
            }
        }
    }
    const Pack<double, L> un = ldp<double, L>(a.u_n + base);
    Pack<double, L> uo;
    Pack<float, L> u32;
#pragma unroll
    for (int j = 0; j < L; j++) {
        uo.v[j] = un.v[j] + a.dts * ((double)adv[j] + pgf[j]);
        u32.v[j] = (float)uo.v[j];
    }
    stp<double, L>(a.u_o + base, uo);
    if (a.u32_o) stp<float, L>(a.u32_o + base, u32);
}

// ---------------------------------------------------------------------------
// shadows: FP32 copies of u and theta for the mixed policy
// ---------------------------------------------------------------------------
template <int MODEL>
__global__ void k_shadows(StageArgs a) {
    const int KM = a.K * a.M;
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long nE = (long)a.mesh.E * KM, nC = (long)a.mesh.N * KM;
    if (idx < nE) a.u32_o[idx] = (float)a.u_o[idx];
    if (MODEL != MODEL_SW && a.th32_o && idx < nC) {
        const int i = (int)(idx / KM);
        const int km = (int)(idx - (long)i * KM);
        const int k = km / a.M, mm = km - k * a.M;
        a.th32_o[idx] = (float)(a.Th_o[idx] / layer_mass<MODEL>(a, k, a.ps_o[(long)i * a.M + mm]));
    }
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
namespace {
inline unsigned nblocks(long n, int b) { return (unsigned)((n + b - 1) / b); }
// values per lane of the edge kernel: 2 when the (k, m) pairs split evenly
inline int edge_values_per_lane(int K, int M) { return (M == 1 ? (K % 2 == 0) : (M % 2 == 0)) ? 2 : 1; }

template <int MODEL, typename R>
hipError_t launch_stage_t(const StageArgs &a, int which, hipStream_t s) {
    const int KM = a.K * a.M;
    const int colthreads = a.cpb * KM;
    const unsigned colblocks = nblocks(a.mesh.N, a.cpb);
    const int fb = a.flat_block;
    size_t lds_a = (size_t)a.cpb * KM * sizeof(double);
    if (MODEL == MODEL_NDC) lds_a += (size_t)a.cpb * (a.K + 1) * a.M * sizeof(double);
    size_t lds_b = (size_t)a.cpb * KM * sizeof(double);
    if (MODEL == MODEL_NDC) lds_b = (size_t)a.cpb * (9 * KM + (a.K + 1) * a.M + KM) * sizeof(double);
    switch (which) {
    case KERNEL_CELL_A:
        hipLaunchKernelGGL((k_cell_a<MODEL, R>), dim3(colblocks), dim3(colthreads), lds_a, s, a);
        break;
    case KERNEL_VERTEX:
        hipLaunchKernelGGL((k_vertex<MODEL, R>), dim3(nblocks((long)a.mesh.V * KM, fb)), dim3(fb), 0, s, a);
        break;
    case KERNEL_CELL_B:
        if (MODEL == MODEL_SW) return hipSuccess;
        hipLaunchKernelGGL((k_cell_b<MODEL, R>), dim3(colblocks), dim3(colthreads), lds_b, s, a);
        break;
    case KERNEL_EDGE: {
        const int L = edge_values_per_lane(a.K, a.M);
        const long n = (long)a.mesh.E * (KM / L);
        const bool one = (a.M == 1);
        if (L == 2 && one)
            hipLaunchKernelGGL((k_edge<MODEL, R, 2, true>), dim3(nblocks(n, fb)), dim3(fb), 0, s, a);
        else if (L == 2)
            hipLaunchKernelGGL((k_edge<MODEL, R, 2, false>), dim3(nblocks(n, fb)), dim3(fb), 0, s, a);
        else if (one)
            hipLaunchKernelGGL((k_edge<MODEL, R, 1, true>), dim3(nblocks(n, fb)), dim3(fb), 0, s, a);
        else
            hipLaunchKernelGGL((k_edge<MODEL, R, 1, false>), dim3(nblocks(n, fb)), dim3(fb), 0, s, a);
        break;
    }
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
}  // namespace

size_t stage_lds_bytes(int model, int which, int cpb, int K, int M) {
    const size_t KM = (size_t)K * M;
    if (which == KERNEL_CELL_A) return cpb * KM * 8 + (model == MODEL_NDC ? cpb * (K + 1) * (size_t)M * 8 : 0);
    if (which == KERNEL_CELL_B) return model == MODEL_NDC ? cpb * (10 * KM + (K + 1) * (size_t)M) * 8 : cpb * KM * 8;
    return 0;
}

hipError_t launch_stage_kernel(int model, int policy, const StageArgs &a, int which, hipStream_t s) {
    if (policy == POLICY_DBL) {
        if (model == MODEL_SW) return launch_stage_t<MODEL_SW, double>(a, which, s);
        if (model == MODEL_HDC) return launch_stage_t<MODEL_HDC, double>(a, which, s);
        return launch_stage_t<MODEL_NDC, double>(a, which, s);
    }
    if (model == MODEL_SW) return launch_stage_t<MODEL_SW, float>(a, which, s);
    if (model == MODEL_HDC) return launch_stage_t<MODEL_HDC, float>(a, which, s);
    return launch_stage_t<MODEL_NDC, float>(a, which, s);
}

hipError_t launch_shadows(int model, const StageArgs &a, hipStream_t s) {
    const long n = (long)(a.mesh.E > a.mesh.N ? a.mesh.E : a.mesh.N) * a.K * a.M;
    if (model == MODEL_SW) hipLaunchKernelGGL(k_shadows<MODEL_SW>, dim3(nblocks(n, 256)), dim3(256), 0, s, a);
    else if (model == MODEL_HDC) hipLaunchKernelGGL(k_shadows<MODEL_HDC>, dim3(nblocks(n, 256)), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_shadows<MODEL_NDC>, dim3(nblocks(n, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace mpdc
