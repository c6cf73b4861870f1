// sph_adjoint.hip -- reverse-mode kernels of the SPH step (adjoint of the
// density update, wall pressure and pair sweeps) and their C ABI.
//
// The forward step n (Sec. 2.6) maps the sorted state at r^n to r^{n+1}:
//   sigma, rho~ = R(sigma, rho^n)                     Eqs. (4), (17)
//   v^{n+1/2} = v^n + dt/2 a^n,  r^{n+1} = r^n + dt v  Eqs. (19), (20)
//   p_w = PW(r^{n+1}, rho~)                            Eq. (12)
//   rho^{n+1} = rho~ + dt D(r^{n+1}, v, rho~, p_w)     Eqs. (9), (21)
//   A = MOM(r^{n+1}, v, rho^{n+1}, p_w), v^{n+1} = v + dt/2 A   Eqs. (10), (22)
// The kernels below apply the transposed Jacobians in the reverse order.
// Each pair sum is transposed by a gather in the particle's own loop (the
// neighbour relation is symmetric), so no floating-point atomics are used.
// Parameter derivatives go through per-block partial sums reduced in a
// fixed order.  All adjoint arithmetic is FP64; the forward state is read
// in its own precision T.
//
// Pair notation: d = r_i - r_j, r = |d|, t = 1 - r/(2h), F = W'(r)/r =
// gfac t^3, F' = dF/dr = -1.5 gfac t^2 / h, C = m F/(rho_i rho_j).
// Momentum (fluid pair): f_ij = C [V(r) v_ij - 2 p* d] with V = 2 mu r^2/
// (r^2 + eta^2), U_L - U_R = J = -(v_ij . d)/r, beta = min(3 max(J,0), c),
// p* = (rho_i p_j + rho_j p_i + rho_i rho_j beta J)/(rho_i + rho_j).  Since
// f_ji = -f_ij, the pair's share of sum_i Abar_i . A_i is
// (Abar_i - Abar_j) . f_ij: one derivative evaluation per pair and side.
// Continuity: D_i = 2 m rho_i sum_j G_ij with G_ij = F [rho_j u + (p_i -
// p_j) r/c]/(rho_j (rho_i + rho_j)), u = v_ij . d; with psi_i = 2 m
// kappa_i rho_i (kappa = dt rhobar^{n+1}) the pair's share is
// (F/S) [(psi_i + psi_j) u + (psi_i/rho_j - psi_j/rho_i)(p_i - p_j) r/c].
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "sph.h"
#include "sph_device.h"
#include "sph_host.h"

using namespace sph;

namespace {

constexpr int kNth = SPH_NTHETA;

// FP64 run constants of the adjoint.
struct AdjPar {
    double h, alpha, gfac, m, rho0, c, c2, mu, eta2, gamma_p, dx, dt, half_dt, sigma0;
    double g[3], gw[3];
    int penalty;
};

// Run constants at step `step` (the time of the state being reversed): in
// a moving tank Eq. (12) takes g - a_w - X''(t) there.
AdjPar make_adj(const sph_desc* d, int64_t step = 0) {
    AdjPar Q;
    const double h = d->h;
    Q.h = h;
    Q.alpha = d->dim == 2 ? 7.0 / (4.0 * M_PI * h * h) : 21.0 / (16.0 * M_PI * h * h * h);
    Q.gfac = -5.0 * Q.alpha / (h * h);
    Q.m = d->rho0 * (d->dim == 2 ? d->dx * d->dx : d->dx * d->dx * d->dx);
    Q.rho0 = d->rho0;
    Q.c = d->c0;
    Q.c2 = d->c0 * d->c0;
    Q.mu = d->mu;
    Q.eta2 = 0.01 * h * h;
    Q.gamma_p = d->gamma_p;
    Q.dx = d->dx;
    Q.dt = d->dt;
    Q.half_dt = 0.5 * d->dt;
    Q.sigma0 = d->sigma0;
    const Motion mo = motion_at(d, step);
    for (int k = 0; k < 3; ++k) {
        Q.g[k] = d->g[k];
        Q.gw[k] = d->g[k] - d->a_wall[k] - mo.A[k];
    }
    Q.penalty = d->penalty_all ? 1 : 0;
    return Q;
}

NbrMask fmask(const uint64_t* m, const int32_t* c, int64_t n) {
    return (m && c) ? NbrMask{m, c, n} : NbrMask{nullptr, nullptr, 0};
}

struct PairGeo {
    double d[3], r2, r, t, F, Fpr, W;  // Fpr = F'(r)/r
};

template <int D, typename T>
__device__ __forceinline__ PairGeo geo(const AdjPar& Q, const T dT[3]) {
    PairGeo g;
    g.r2 = 0.0;
    for (int k = 0; k < 3; ++k) {
        g.d[k] = k < D ? (double)dT[k] : 0.0;
        g.r2 += g.d[k] * g.d[k];
    }
    g.r = sqrt(g.r2);
    g.t = 1.0 - 0.5 * g.r / Q.h;
    const double t2 = g.t * g.t;
    g.F = Q.gfac * t2 * g.t;
    g.Fpr = (-1.5 * Q.gfac * t2 / Q.h) / g.r;
    g.W = Q.alpha * t2 * t2 * (1.0 + 2.0 * g.r / Q.h);
    return g;
}

template <int D>
__device__ __forceinline__ double dotv(const double* a, const double* b) {
    double s = 0.0;
    for (int k = 0; k < D; ++k) s += a[k] * b[k];
    return s;
}

// Block sum of kNth values into part[block * kNth + k] (fixed order).
__device__ __forceinline__ void block_partials(const double v[kNth], double* part) {
    __shared__ double red[kNth][kBlock];
    for (int k = 0; k < kNth; ++k) red[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int k = 0; k < kNth; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x < kNth) part[(int64_t)blockIdx.x * kNth + threadIdx.x] = red[threadIdx.x][0];
}

// Abar = ab + ha vb of every particle in a frame's sorted order (the pair
// sweeps read it by neighbour index).
__global__ void __launch_bounds__(kBlock)
    k_gather_abar(int dim, int64_t nf, const int32_t* __restrict__ pid, const double* __restrict__ ab,
                  const double* __restrict__ vb, double ha, double* __restrict__ abar) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nf) return;
    const int64_t p = pid[i];
    for (int k = 0; k < dim; ++k) abar[k * nf + i] = ab[k * nf + p] + (vb ? ha * vb[k * nf + p] : 0.0);
}

__global__ void k_theta_reduce(const double* __restrict__ part, int nblocks, double* __restrict__ theta) {
    __shared__ double red[kNth][kBlock];
    double v[kNth] = {0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblocks; b += kBlock)
        for (int k = 0; k < kNth; ++k) v[k] += part[(int64_t)b * kNth + k];
    for (int k = 0; k < kNth; ++k) red[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int k = 0; k < kNth; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x < kNth) theta[threadIdx.x] += red[threadIdx.x][0];
}

// Limiter of Eq. (8): beta = min(3 max(J, 0), c), with dbeta/dJ and
// dbeta/dc (max' = 0 at 0; on a tie of min the 3 max(J, 0) branch).
__device__ __forceinline__ void limiter(double J, double c, double& beta, double& bJ, double& bc) {
    const double jp = J > 0.0 ? J : 0.0;
    if (3.0 * jp <= c) {
        beta = 3.0 * jp;
        bJ = J > 0.0 ? 3.0 : 0.0;
        bc = 0.0;
    } else {
        beta = c;
        bJ = 0.0;
        bc = 1.0;
    }
}

// ---------------------------------------------------------------------------
// Momentum backward (fluid side).  Abar_i = ab_i + ha vb_i (the second kick
// v^{n+1} = v + dt/2 A and a^{n+1} = A).  Writes
//   xb  += dL/dr,  vh_out = vb + dL/dv,  rp_out = rho_in + dL/drho.
// ---------------------------------------------------------------------------
template <typename T, int D>
__global__ void __launch_bounds__(kBlock)
    k_mom_bwd(Par<T> P, AdjPar Q, NbrMask LF, NbrMask LW, int64_t nf, int64_t nw, const int32_t* __restrict__ key,
              const int32_t* __restrict__ pid, const T* __restrict__ off,
              const int32_t* __restrict__ fstart, const T* __restrict__ vh,
              const T* __restrict__ rp, const int32_t* __restrict__ wkey,
              const T* __restrict__ woff, const int32_t* __restrict__ wstart,
              const T* __restrict__ pw, const T* __restrict__ nrm, const double* __restrict__ ab,
              const double* __restrict__ vb, double ha, const double* __restrict__ abar,
              const double* __restrict__ rho_in, double* __restrict__ xb, double* __restrict__ vh_out,
              double* __restrict__ rp_out, double* __restrict__ rp_out_s, double* __restrict__ part) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double th[kNth] = {0, 0, 0, 0};
    if (i < nf) {
        const int64_t p = pid[i];
        int c[3];
        cell_of(P, key[i], c);
        const T oi[3] = {off[i], off[nf + i], D == 3 ? off[2 * nf + i] : T(0)};
        double vi[3] = {0, 0, 0}, Ai[3] = {0, 0, 0};
        for (int k = 0; k < D; ++k) {
            vi[k] = (double)vh[k * nf + i];
            Ai[k] = ab[k * nf + p] + (vb ? ha * vb[k * nf + p] : 0.0);
        }
        const double ri = Q.rho0 + (double)rp[i];
        const double pi_ = Q.c2 * (double)rp[i];
        double gx[3] = {0, 0, 0}, gv[3] = {0, 0, 0}, gr = 0.0;
        visit<T, D>(P, LF, i, fstart, off, off + nf, off + 2 * nf, c, oi,
                    [&](int j, const T dT[3], T r2T, uint32_t) {
            if (!(r2T > T(0))) return;
            const PairGeo G = geo<D>(Q, dT);
            double vj[3] = {0, 0, 0}, dA[3] = {0, 0, 0}, dv[3] = {0, 0, 0};
            for (int k = 0; k < D; ++k) {
                vj[k] = (double)vh[k * nf + j];
                dA[k] = Ai[k] - abar[k * nf + j];  // j's Abar, gathered into this frame's order
                dv[k] = vi[k] - vj[k];
            }
            const double rj = Q.rho0 + (double)rp[j];
            const double pj_ = Q.c2 * (double)rp[j];
            const double u = dotv<D>(dv, G.d);
            const double J = -u / G.r;
            double beta, bJ, bc;
            limiter(J, Q.c, beta, bJ, bc);
            const double S = ri + rj;
            const double ps = (ri * pj_ + rj * pi_ + ri * rj * beta * J) / S;
            const double psJ = ri * rj * (beta + J * bJ) / S;
            const double psRi = (pj_ + rj * Q.c2 + rj * beta * J - ps) / S;
            const double Cm = Q.m / (ri * rj);
            const double C = Cm * G.F;
            const double den = G.r2 + Q.eta2;
            const double V = 2.0 * Q.mu * G.r2 / den;
            const double Vd = 4.0 * Q.mu * Q.eta2 / (den * den);
            const double Vmu = 2.0 * G.r2 / den;
            const double a = dotv<D>(dA, G.d), b = dotv<D>(dA, dv);
            const double Lin = V * b - 2.0 * ps * a;
            for (int k = 0; k < D; ++k) {
                const double Jd = -dv[k] / G.r - J * G.d[k] / G.r2;
                gx[k] += Cm * G.Fpr * Lin * G.d[k] +
                         C * (Vd * b * G.d[k] - 2.0 * a * psJ * Jd - 2.0 * ps * dA[k]);
                gv[k] += C * (V * dA[k] + 2.0 * a * psJ * G.d[k] / G.r);
            }
            gr += -(C / ri) * Lin - 2.0 * C * a * psRi;
            // own share Abar_i . f_ij for the parameters
            const double ai = dotv<D>(Ai, G.d), bi = dotv<D>(Ai, dv);
            th[SPH_THETA_MU] += C * Vmu * bi;
            const double Nc = 2.0 * (ri * pj_ + rj * pi_) / Q.c + ri * rj * J * bc;
            th[SPH_THETA_C0] += -2.0 * C * ai * Nc / S;
        });
        if (nw > 0 && (!LW.mask || LW.count[i] != 0))  // no wall neighbour: nothing to add
            visit<T, D>(P, LW, i, wstart, woff, woff + nw, woff + 2 * nw, c, oi,
                        [&](int w, const T dT[3], T r2T, uint32_t) {
                if (!(r2T > T(0))) return;
                const PairGeo G = geo<D>(Q, dT);
                const double pwv = (double)pw[w];
                const double rw = Q.rho0 + pwv / Q.c2;
                const double Sw = ri + rw;
                const double Cm = Q.m / (ri * rw);
                const double C = Cm * G.F;
                const double ps = (ri * pwv + rw * pi_) / Sw;
                const double den = G.r2 + Q.eta2;
                const double V = 2.0 * Q.mu * G.r2 / den;
                const double Vd = 4.0 * Q.mu * Q.eta2 / (den * den);
                const double Vmu = 2.0 * G.r2 / den;
                double n[3] = {0, 0, 0};
                double pen = 0.0, pen_g = 0.0, pen_ds = 0.0, pen_r = 0.0;
                if (Q.penalty) {
                    for (int k = 0; k < D; ++k) n[k] = (double)nrm[k * nw + w];
                    const double proj = dotv<D>(G.d, n);
                    const double ap = fabs(proj);
                    const double delta = 2.0 * ap / Q.dx;
                    if (delta < 1.0) {
                        const double om = 1.0 - delta;
                        const double api = fabs(pi_);
                        const double sp = proj > 0.0 ? 1.0 : (proj < 0.0 ? -1.0 : 0.0);
                        const double spi = pi_ > 0.0 ? 1.0 : (pi_ < 0.0 ? -1.0 : 0.0);
                        pen_g = -2.0 * om * om * api * ap;
                        pen = Q.gamma_p * pen_g;
                        pen_ds = -2.0 * Q.gamma_p * api * om * (1.0 - 3.0 * delta) * sp;
                        pen_r = -2.0 * Q.gamma_p * om * om * ap * spi * Q.c2;
                    }
                }
                const double a = dotv<D>(Ai, G.d), b = dotv<D>(Ai, vi), e = dotv<D>(Ai, n);
                const double Lin = V * b - 2.0 * ps * a + pen * e;
                for (int k = 0; k < D; ++k) {
                    gx[k] += Cm * G.Fpr * Lin * G.d[k] +
                             C * (Vd * b * G.d[k] - 2.0 * ps * Ai[k] + e * pen_ds * n[k]);
                    gv[k] += C * V * Ai[k];
                }
                const double psR = (pwv + rw * Q.c2 - ps) / Sw;
                gr += -(C / ri) * Lin + C * (-2.0 * a * psR + e * pen_r);
                th[SPH_THETA_MU] += C * Vmu * b;
                th[SPH_THETA_GAMMA] += C * pen_g * e;
                const double rwc = -2.0 * pwv / (Q.c2 * Q.c);
                const double Cc = -C * rwc / rw;
                const double Nwc = rwc * pi_ + rw * 2.0 * pi_ / Q.c;
                const double psc = (Nwc - ps * rwc) / Sw;
                th[SPH_THETA_C0] += Cc * Lin + C * (-2.0 * a * psc + e * 2.0 * pen / Q.c);
            });
        for (int k = 0; k < D; ++k) {
            xb[k * nf + p] += gx[k];
            vh_out[k * nf + p] = (vb ? vb[k * nf + p] : 0.0) + gv[k];
        }
        const double rpv = (rho_in ? rho_in[p] : 0.0) + gr;
        rp_out[p] = rpv;
        if (rp_out_s) rp_out_s[i] = rpv;
    }
    block_partials(th, part);
}

// ---------------------------------------------------------------------------
// Continuity backward (fluid side): kappa_i = dt rpb_i (adjoint of drho/dt),
// psi_i = 2 m kappa_i rho~_i.  Writes xb += , vhb += ,
// rtb = rpb + d/drho~ (identity of Eq. (21) plus the sweep).
// ---------------------------------------------------------------------------
template <typename T, int D>
__global__ void __launch_bounds__(kBlock)
    k_cont_bwd(Par<T> P, AdjPar Q, NbrMask LF, NbrMask LW, int64_t nf, int64_t nw, const int32_t* __restrict__ key,
               const int32_t* __restrict__ pid, const T* __restrict__ off,
               const int32_t* __restrict__ fstart, const T* __restrict__ vh,
               const T* __restrict__ rt, const T* __restrict__ woff,
               const int32_t* __restrict__ wstart, const T* __restrict__ pw,
               const double* __restrict__ rpb, const double* __restrict__ rpbs, double* __restrict__ xb,
               double* __restrict__ vhb, double* __restrict__ rtb, double* __restrict__ part) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double th[kNth] = {0, 0, 0, 0};
    if (i < nf) {
        const int64_t p = pid[i];
        int c[3];
        cell_of(P, key[i], c);
        const T oi[3] = {off[i], off[nf + i], D == 3 ? off[2 * nf + i] : T(0)};
        double vi[3] = {0, 0, 0};
        for (int k = 0; k < D; ++k) vi[k] = (double)vh[k * nf + i];
        const double ri = Q.rho0 + (double)rt[i];
        const double kap = Q.dt * rpb[p];
        const double psi_i = 2.0 * Q.m * kap * ri;
        double gx[3] = {0, 0, 0}, gv[3] = {0, 0, 0}, gr = 0.0, sumG = 0.0;
        visit<T, D>(P, LF, i, fstart, off, off + nf, off + 2 * nf, c, oi,
                    [&](int j, const T dT[3], T r2T, uint32_t) {
            if (!(r2T > T(0))) return;
            const PairGeo G = geo<D>(Q, dT);
            const double rj = Q.rho0 + (double)rt[j];
            const double psi_j = 2.0 * Q.m * Q.dt * rpbs[j] * rj;
            double dv[3] = {0, 0, 0};
            for (int k = 0; k < D; ++k) dv[k] = vi[k] - (double)vh[k * nf + j];
            const double u = dotv<D>(dv, G.d);
            const double dp = Q.c2 * ((double)rt[i] - (double)rt[j]);
            const double S = ri + rj;
            const double Phi = psi_i + psi_j;
            const double Psi = psi_i / rj - psi_j / ri;
            const double inner = Phi * u + Psi * dp * G.r / Q.c;
            const double L = G.F / S * inner;
            sumG += G.F * (rj * u + dp * G.r / Q.c) / (rj * S);
            for (int k = 0; k < D; ++k) {
                gx[k] += G.Fpr * G.d[k] / S * inner + G.F / S * (Phi * dv[k] + Psi * dp / Q.c * G.d[k] / G.r);
                gv[k] += G.F / S * Phi * G.d[k];
            }
            gr += -L / S + G.F / S * (G.r / Q.c) * (psi_j / (ri * ri) * dp + Psi * Q.c2);
            th[SPH_THETA_C0] += psi_i * G.F * dp * G.r / (rj * S * Q.c2);
        });
        if (nw > 0 && (!LW.mask || LW.count[i] != 0))  // no wall neighbour: nothing to add
            visit<T, D>(P, LW, i, wstart, woff, woff + nw, woff + 2 * nw, c, oi,
                        [&](int w, const T dT[3], T r2T, uint32_t) {
                if (!(r2T > T(0))) return;
                const PairGeo G = geo<D>(Q, dT);
                const double pwv = (double)pw[w];
                const double rw = Q.rho0 + pwv / Q.c2;
                const double Sw = ri + rw;
                const double pi_ = Q.c2 * (double)rt[i];
                const double uw = dotv<D>(vi, G.d);
                const double E = rw * uw + (pi_ - pwv) * G.r / Q.c;
                sumG += G.F * E / (rw * Sw);
                for (int k = 0; k < D; ++k) {
                    gx[k] += psi_i / (rw * Sw) *
                             (G.Fpr * G.d[k] * E + G.F * (rw * vi[k] + (pi_ - pwv) / Q.c * G.d[k] / G.r));
                    gv[k] += psi_i * G.F * G.d[k] / Sw;
                }
                gr += psi_i * G.F / rw * (Q.c * G.r / Sw - E / (Sw * Sw));
                const double rwc = -2.0 * pwv / (Q.c2 * Q.c);
                const double Ec = rwc * uw + (2.0 * pi_ / Q.c) * G.r / Q.c - (pi_ - pwv) * G.r / Q.c2;
                const double q = rw * Sw;
                th[SPH_THETA_C0] += psi_i * G.F * (Ec / q - E * (rwc * Sw + rw * rwc) / (q * q));
            });
        for (int k = 0; k < D; ++k) {
            xb[k * nf + p] += gx[k];
            vhb[k * nf + p] += gv[k];
        }
        rtb[p] = rpb[p] + 2.0 * Q.m * kap * sumG + gr;
    }
    block_partials(th, part);
}

// ---------------------------------------------------------------------------
// Wall side: pbar_w = d/dp_w of the momentum and continuity sweeps (+ the
// probe's dt/n_probe), then lam_w = pbar_w / sum_f W_wf for Eq. (12).
// ---------------------------------------------------------------------------
template <typename T, int D>
__global__ void __launch_bounds__(kBlock)
    k_wall_bwd(Par<T> P, AdjPar Q, NbrMask LWF, int64_t nf, int64_t nw, const int32_t* __restrict__ wkey,
               const int32_t* __restrict__ wpid, const T* __restrict__ woff,
               const T* __restrict__ nrm, const T* __restrict__ pw, const int32_t* __restrict__ pid,
               const T* __restrict__ off, const int32_t* __restrict__ fstart,
               const T* __restrict__ vh, const T* __restrict__ rp, const T* __restrict__ rt,
               const double* __restrict__ abar, const double* __restrict__ rpbs,
               const int32_t* __restrict__ probe, int np, double* __restrict__ lam) {
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= nw) return;
    int c[3];
    cell_of(P, wkey[w], c);
    const T ow[3] = {woff[w], woff[nw + w], D == 3 ? woff[2 * nw + w] : T(0)};
    const double pwv = (double)pw[w];
    const double rw = Q.rho0 + pwv / Q.c2;
    double n[3] = {0, 0, 0};
    if (Q.penalty)
        for (int k = 0; k < D; ++k) n[k] = (double)nrm[k * nw + w];
    double SW = 0.0, pbar = 0.0;
    if (nf > 0)
        visit<T, D>(P, LWF, w, fstart, off, off + nf, off + 2 * nf, c, ow,
                    [&](int f, const T dT[3], T r2T, uint32_t) {
            const PairGeo G0 = geo<D>(Q, dT);
            SW += G0.W;
            if (!(r2T > T(0))) return;
            double dfw[3] = {0, 0, 0}, vf[3] = {0, 0, 0};
            for (int k = 0; k < D; ++k) {
                dfw[k] = -G0.d[k];
                vf[k] = (double)vh[k * nf + f];
            }
            // momentum: fluid f sees this wall with p* of Eq. (11), viscous, penalty
            if (abar) {
                double Af[3] = {0, 0, 0};
                for (int k = 0; k < D; ++k) Af[k] = abar[k * nf + f];  // f's Abar in this frame's order
                const double rf = Q.rho0 + (double)rp[f];
                const double pf_ = Q.c2 * (double)rp[f];
                const double Sw = rf + rw;
                const double C = Q.m * G0.F / (rf * rw);
                const double ps = (rf * pwv + rw * pf_) / Sw;
                const double V = 2.0 * Q.mu * G0.r2 / (G0.r2 + Q.eta2);
                double pen = 0.0;
                if (Q.penalty) {
                    const double ap = fabs(dotv<D>(dfw, n));
                    const double delta = 2.0 * ap / Q.dx;
                    if (delta < 1.0) pen = -2.0 * Q.gamma_p * (1.0 - delta) * (1.0 - delta) * fabs(pf_) * ap;
                }
                const double a = dotv<D>(Af, dfw), b = dotv<D>(Af, vf), e = dotv<D>(Af, n);
                const double Lin = V * b - 2.0 * ps * a + pen * e;
                const double Cpw = -C / (rw * Q.c2);
                const double pspw = (rf + pf_ / Q.c2 - ps / Q.c2) / Sw;
                pbar += Cpw * Lin - 2.0 * C * a * pspw;
            }
            // continuity: psi_f G_fw with the reinitialised density
            if (rpbs) {
                const double rf = Q.rho0 + (double)rt[f];
                const double pf_ = Q.c2 * (double)rt[f];
                const double psi = 2.0 * Q.m * Q.dt * rpbs[f] * rf;
                const double Sw = rf + rw;
                const double uw = dotv<D>(vf, dfw);
                const double E = rw * uw + (pf_ - pwv) * G0.r / Q.c;
                const double Epw = uw / Q.c2 - G0.r / Q.c;
                const double q = rw * Sw;
                pbar += psi * G0.F * (Epw / q - E * (Sw + rw) / (Q.c2 * q * q));
            }
        });
    if (probe) {
        const int32_t id = wpid[w];
        for (int a = 0; a < np; ++a)
            if (probe[a] == id) pbar += Q.dt / (double)np;
    }
    lam[w] = SW > 0.0 ? pbar / SW : 0.0;
}

// ---------------------------------------------------------------------------
// Wall pressure backward (fluid side): with lam_w = pbar_w / sum W,
// dp_w/dr_f and dp_w/drho_f of Eq. (12) (e = r_w - r_f).
// ---------------------------------------------------------------------------
template <typename T, int D>
__global__ void __launch_bounds__(kBlock)
    k_pw_bwd(Par<T> P, AdjPar Q, NbrMask LW, int64_t nf, int64_t nw, const int32_t* __restrict__ key,
             const int32_t* __restrict__ pid, const T* __restrict__ off,
             const T* __restrict__ rho, const T* __restrict__ woff,
             const int32_t* __restrict__ wstart, const T* __restrict__ pw,
             const double* __restrict__ lam, double* __restrict__ xb, double* __restrict__ rhob,
             double* __restrict__ part) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double th[kNth] = {0, 0, 0, 0};
    if (i < nf && nw > 0) {
        const int64_t p = pid[i];
        int c[3];
        cell_of(P, key[i], c);
        const T oi[3] = {off[i], off[nf + i], D == 3 ? off[2 * nf + i] : T(0)};
        const double rf = Q.rho0 + (double)rho[i];
        const double pf_ = Q.c2 * (double)rho[i];
        double gx[3] = {0, 0, 0}, gr = 0.0;
        if (!LW.mask || LW.count[i] != 0)  // no wall neighbour: nothing to add
        visit<T, D>(P, LW, i, wstart, woff, woff + nw, woff + 2 * nw, c, oi,
                    [&](int w, const T dT[3], T r2T, uint32_t) {
            const double lw = lam[w];
            if (lw == 0.0) return;
            const PairGeo G = geo<D>(Q, dT);
            double e[3] = {0, 0, 0};
            for (int k = 0; k < D; ++k) e[k] = -G.d[k];
            const double ge = dotv<D>(Q.gw, e);
            const double pwv = (double)pw[w];
            if (r2T > T(0))
                for (int k = 0; k < D; ++k)
                    gx[k] += lw * ((pf_ - pwv) * G.F * G.d[k] - rf * (Q.gw[k] * G.W + ge * G.F * e[k]));
            else
                for (int k = 0; k < D; ++k) gx[k] += -lw * rf * Q.gw[k] * G.W;
            gr += lw * G.W * (Q.c2 + ge);
            th[SPH_THETA_C0] += lw * 2.0 * pf_ * G.W / Q.c;
        });
        for (int k = 0; k < D; ++k) xb[k * nf + p] += gx[k];
        rhob[p] += gr;
    }
    block_partials(th, part);
}

// ---------------------------------------------------------------------------
// Drift, half kick and Eq. (17), transposed (elementwise, frame n order):
//   vhb += dt xb;  vb = vhb;  ab = dt/2 vhb;  sigb, rhob from rtb.
// ---------------------------------------------------------------------------
template <typename T, int D>
__global__ void __launch_bounds__(kBlock)
    k_kick_reinit_bwd(Par<T> P, AdjPar Q, int64_t nf, const int32_t* __restrict__ pid,
                      const T* __restrict__ sigma, const T* __restrict__ rho,
                      const double* __restrict__ xb, const double* __restrict__ vhb,
                      const double* __restrict__ rtb, double* __restrict__ vb,
                      double* __restrict__ ab, double* __restrict__ sigbs, double* __restrict__ rhob) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nf) return;
    const int64_t p = pid[i];
    for (int k = 0; k < D; ++k) {
        const double v = vhb[k * nf + p] + Q.dt * xb[k * nf + p];
        vb[k * nf + p] = v;
        ab[k * nf + p] = Q.half_dt * v;
    }
    // the branch of max(0, rho* - rho_s) exactly as the forward took it (in T)
    const T s = sigma[i];
    const T drs = P.rho0_over_sigma0 * (s - P.sigma0);
    const T dstar = rho[i];
    const bool excess = dstar - drs > T(0);
    const double rstar = Q.rho0 + (double)dstar;
    const double rs = Q.rho0 * (double)s / Q.sigma0;
    const double Rs = excess ? (Q.rho0 / Q.sigma0) * (1.0 - Q.rho0 / rstar) : Q.rho0 / Q.sigma0;
    const double Rr = excess ? Q.rho0 * rs / (rstar * rstar) : 0.0;
    sigbs[i] = Rs * rtb[p];  // this frame's order: the number density sweep reads it by neighbour
    rhob[p] = Rr * rtb[p];
}

// Number density backward at r^n: xb_i += sum_j (sigb_i + sigb_j) F d + sum_w sigb_i F d.
template <typename T, int D>
__global__ void __launch_bounds__(kBlock)
    k_sigma_bwd(Par<T> P, AdjPar Q, NbrMask LF, NbrMask LW, int64_t nf, int64_t nw, const int32_t* __restrict__ key,
                const int32_t* __restrict__ pid, const T* __restrict__ off,
                const int32_t* __restrict__ fstart, const T* __restrict__ woff,
                const int32_t* __restrict__ wstart, const double* __restrict__ sigbs,
                double* __restrict__ xb) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nf) return;
    const int64_t p = pid[i];
    int c[3];
    cell_of(P, key[i], c);
    const T oi[3] = {off[i], off[nf + i], D == 3 ? off[2 * nf + i] : T(0)};
    const double si = sigbs[i];
    double gx[3] = {0, 0, 0};
    visit<T, D>(P, LF, i, fstart, off, off + nf, off + 2 * nf, c, oi,
                [&](int j, const T dT[3], T r2T, uint32_t) {
        if (!(r2T > T(0))) return;
        const PairGeo G = geo<D>(Q, dT);
        const double s = si + sigbs[j];
        for (int k = 0; k < D; ++k) gx[k] += s * G.F * G.d[k];
    });
    if (nw > 0 && (!LW.mask || LW.count[i] != 0))  // no wall neighbour: nothing to add
        visit<T, D>(P, LW, i, wstart, woff, woff + nw, woff + 2 * nw, c, oi,
                    [&](int, const T dT[3], T r2T, uint32_t) {
            if (!(r2T > T(0))) return;
            const PairGeo G = geo<D>(Q, dT);
            for (int k = 0; k < D; ++k) gx[k] += si * G.F * G.d[k];
        });
    for (int k = 0; k < D; ++k) xb[k * nf + p] += gx[k];
}

// Initial state: z = s z_ref (s = H / H_ref) and rho = rho0 (1 + g (H - z)/c^2)
// with z above the floor at 0: dJ/dH = sum xb_z z/H + rhob rho0 g (H - z)/(c^2 H),
// dJ/dc0 += sum rhob (-2 rho0 g (H - z)/c^3).
template <typename T, int D>
__global__ void __launch_bounds__(kBlock)
    k_init_theta(Par<T> P, AdjPar Q, GridD Gd, double H, int64_t nf, const int32_t* __restrict__ key,
                 const int32_t* __restrict__ pid, const T* __restrict__ off,
                 const double* __restrict__ xb, const double* __restrict__ rhob,
                 double* __restrict__ part) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double th[kNth] = {0, 0, 0, 0};
    if (i < nf) {
        const int64_t p = pid[i];
        int c[3];
        cell_of(P, key[i], c);
        const int kz = D - 1;
        const double z = Gd.lo[kz] + (double)c[kz] * Gd.L + (double)off[(int64_t)kz * nf + i];
        const double gmag = fabs(Q.g[kz]);
        th[SPH_THETA_H] = xb[(int64_t)kz * nf + p] * z / H + rhob[p] * Q.rho0 * gmag * (H - z) / (Q.c2 * H);
        th[SPH_THETA_C0] = rhob[p] * (-2.0 * Q.rho0 * gmag * (H - z) / (Q.c2 * Q.c));
    }
    block_partials(th, part);
}

__global__ void k_zero_f64(double* __restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

struct AdjWork {
    double* vhb;   // [dim][nf]
    double* rpb;   // [nf]
    double* rtb;   // [nf]
    double* sigb;  // [nf] number density adjoint, in the sorted order of the frame being reversed
    double* abar;  // [dim][nf] Abar = ab + dt/2 vb, in the frame's sorted order
    double* rpbs;  // [nf] rpb in the frame's sorted order
    double* lam;   // [nw]
    double* tmp;   // [dim][nf] discarded velocity adjoint of the initial state
    double* part;  // partial sums, kNth per block
    size_t bytes;
};

AdjWork adj_layout(const sph_desc* d, int64_t nf, int64_t nw, void* base) {
    AdjWork w;
    size_t o = 0;
    char* b = (char*)base;
    auto take = [&](size_t bytes) {
        char* p = b ? b + o : nullptr;
        o += align256(bytes > 0 ? bytes : 1);
        return (double*)p;
    };
    const int64_t nmax = nf > nw ? nf : nw;
    w.vhb = take(sizeof(double) * d->dim * (size_t)nf);
    w.rpb = take(sizeof(double) * (size_t)nf);
    w.rtb = take(sizeof(double) * (size_t)nf);
    w.sigb = take(sizeof(double) * (size_t)nf);
    w.abar = take(sizeof(double) * d->dim * (size_t)nf);
    w.rpbs = take(sizeof(double) * (size_t)nf);
    w.lam = take(sizeof(double) * (size_t)nw);
    w.tmp = take(sizeof(double) * d->dim * (size_t)nf);
    w.part = take(sizeof(double) * kNth * (size_t)((nmax + kBlock - 1) / kBlock + 1));
    w.bytes = o;
    return w;
}

int check_adj(const sph_desc* d, const sph_buffers* b, const sph_adjoint* a) {
    if (d->two_phase) return SPH_ERR_CONFIG;  // the backward covers the single-phase step
    if (!a || !a->theta || !a->work) return SPH_ERR_ARG;
    if (a->work_bytes < sph_adjoint_work_bytes(d, b->n_fluid, b->n_wall)) return SPH_ERR_ARG;
    if (((uintptr_t)a->work & 255) != 0) return SPH_ERR_ARG;
    if (b->n_fluid > 0 && (!a->xb || !a->vb || !a->rhob || !a->ab)) return SPH_ERR_ARG;
    return SPH_OK;
}

int check_frame(const sph_buffers* b, const sph_frame* f, bool need_sigma, bool need_step) {
    if (!f) return SPH_ERR_ARG;
    if (b->n_fluid > 0) {
        if (!f->key || !f->pid || !f->off || !f->fstart || !f->rho) return SPH_ERR_ARG;
        if (need_sigma && !f->sigma) return SPH_ERR_ARG;
        if (need_step && (!f->vh || !f->rt)) return SPH_ERR_ARG;
    }
    if (b->n_wall > 0 && need_step && !f->pw) return SPH_ERR_ARG;
    return SPH_OK;
}

int reduce_theta(const AdjWork& w, int nblocks, double* theta, hipStream_t st) {
    if (nblocks <= 0) return SPH_OK;
    hipLaunchKernelGGL(k_theta_reduce, dim3(1), dim3(kBlock), 0, st, w.part, nblocks, theta);
    SPH_LAUNCH_CHECK();
    return SPH_OK;
}

// Momentum (with the second kick) then continuity, at frame `next`.
template <typename T, int D>
int forces_bwd_t(const sph_desc* d, const sph_buffers* b, const sph_frame* f, sph_adjoint* a,
                 hipStream_t st) {
    const int64_t nf = b->n_fluid, nw = b->n_wall;
    if (nf == 0) return SPH_OK;
    const Par<T> P = make_par<T>(d);
    const AdjPar Q = make_adj(d);
    const AdjWork w = adj_layout(d, nf, nw, a->work);
    const int nb = grid_for(nf);
    hipLaunchKernelGGL(k_gather_abar, dim3(nb), dim3(kBlock), 0, st, D, nf, f->pid, a->ab, a->vb, Q.half_dt,
                       w.abar);
    SPH_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_mom_bwd<T, D>), dim3(nb), dim3(kBlock), 0, st, P, Q, fmask(f->nbr_ff, f->cnt_ff, nf),
                       fmask(f->nbr_fw, f->cnt_fw, nf), nf, nw, f->key, f->pid,
                       (const T*)f->off, f->fstart, (const T*)f->vh, (const T*)f->rho, b->wkey,
                       (const T*)b->woff, b->wstart, (const T*)f->pw, (const T*)b->nrm, a->ab, a->vb,
                       Q.half_dt, (const double*)w.abar, a->rhob, a->xb, w.vhb, w.rpb, w.rpbs, w.part);
    SPH_LAUNCH_CHECK();
    int rc = reduce_theta(w, nb, a->theta, st);
    if (rc) return rc;
    hipLaunchKernelGGL((k_cont_bwd<T, D>), dim3(nb), dim3(kBlock), 0, st, P, Q, fmask(f->nbr_ff, f->cnt_ff, nf),
                       fmask(f->nbr_fw, f->cnt_fw, nf), nf, nw, f->key, f->pid,
                       (const T*)f->off, f->fstart, (const T*)f->vh, (const T*)f->rt, (const T*)b->woff,
                       b->wstart, (const T*)f->pw, w.rpb, (const double*)w.rpbs, a->xb, w.vhb, w.rtb, w.part);
    SPH_LAUNCH_CHECK();
    return reduce_theta(w, nb, a->theta, st);
}

template <typename T, int D>
int wall_bc_bwd_t(const sph_desc* d, const sph_buffers* b, const sph_frame* f, sph_adjoint* a,
                  hipStream_t st) {
    const int64_t nf = b->n_fluid, nw = b->n_wall;
    if (nw == 0) return SPH_OK;
    const Par<T> P = make_par<T>(d);
    const AdjPar Q = make_adj(d, f->nstep);
    const AdjWork w = adj_layout(d, nf, nw, a->work);
    hipLaunchKernelGGL((k_wall_bwd<T, D>), dim3(grid_for(nw)), dim3(kBlock), 0, st, P, Q,
                       fmask(f->nbr_wf, f->cnt_wf, nw), nf, nw,
                       b->wkey, b->wpid, (const T*)b->woff, (const T*)b->nrm, (const T*)f->pw, f->pid,
                       (const T*)f->off, f->fstart, (const T*)f->vh, (const T*)f->rho, (const T*)f->rt,
                       nf > 0 ? (const double*)w.abar : nullptr, nf > 0 ? (const double*)w.rpbs : nullptr,
                       b->n_probe > 0 ? b->probe : nullptr, b->n_probe, w.lam);
    SPH_LAUNCH_CHECK();
    if (nf == 0) return SPH_OK;
    const int nb = grid_for(nf);
    hipLaunchKernelGGL((k_pw_bwd<T, D>), dim3(nb), dim3(kBlock), 0, st, P, Q, fmask(f->nbr_fw, f->cnt_fw, nf),
                       nf, nw, f->key, f->pid,
                       (const T*)f->off, (const T*)f->rt, (const T*)b->woff, b->wstart, (const T*)f->pw,
                       w.lam, a->xb, w.rtb, w.part);
    SPH_LAUNCH_CHECK();
    return reduce_theta(w, nb, a->theta, st);
}

template <typename T, int D>
int density_bwd_t(const sph_desc* d, const sph_buffers* b, const sph_frame* f, sph_adjoint* a,
                  hipStream_t st) {
    const int64_t nf = b->n_fluid, nw = b->n_wall;
    if (nf == 0) return SPH_OK;
    const Par<T> P = make_par<T>(d);
    const AdjPar Q = make_adj(d);
    const AdjWork w = adj_layout(d, nf, nw, a->work);
    const int nb = grid_for(nf);
    hipLaunchKernelGGL((k_kick_reinit_bwd<T, D>), dim3(nb), dim3(kBlock), 0, st, P, Q, nf, f->pid,
                       (const T*)f->sigma, (const T*)f->rho, a->xb, w.vhb, w.rtb, a->vb, a->ab, w.sigb,
                       a->rhob);
    SPH_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_sigma_bwd<T, D>), dim3(nb), dim3(kBlock), 0, st, P, Q, fmask(f->nbr_ff, f->cnt_ff, nf),
                       fmask(f->nbr_fw, f->cnt_fw, nf), nf, nw, f->key, f->pid,
                       (const T*)f->off, f->fstart, (const T*)b->woff, b->wstart, w.sigb, a->xb);
    SPH_LAUNCH_CHECK();
    return SPH_OK;
}

template <typename T, int D>
int init_bwd_t(const sph_desc* d, const sph_buffers* b, const sph_frame* f, double H, sph_adjoint* a,
               hipStream_t st) {
    const int64_t nf = b->n_fluid, nw = b->n_wall;
    if (nf == 0) return SPH_OK;
    const Par<T> P = make_par<T>(d);
    const AdjPar Q = make_adj(d, f->nstep);
    const AdjWork w = adj_layout(d, nf, nw, a->work);
    const int nb = grid_for(nf);
    // a^0 = MOM(r^0, v^0, rho^0, p_w^0): Abar = ab (no kick), rho adjoint in place
    hipLaunchKernelGGL(k_gather_abar, dim3(nb), dim3(kBlock), 0, st, D, nf, f->pid, a->ab, (const double*)nullptr,
                       0.0, w.abar);
    SPH_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_mom_bwd<T, D>), dim3(nb), dim3(kBlock), 0, st, P, Q, fmask(f->nbr_ff, f->cnt_ff, nf),
                       fmask(f->nbr_fw, f->cnt_fw, nf), nf, nw, f->key, f->pid,
                       (const T*)f->off, f->fstart, (const T*)f->vh, (const T*)f->rho, b->wkey,
                       (const T*)b->woff, b->wstart, (const T*)f->pw, (const T*)b->nrm, a->ab,
                       (const double*)nullptr, 0.0, (const double*)w.abar, a->rhob, a->xb, w.tmp, a->rhob,
                       (double*)nullptr, w.part);
    SPH_LAUNCH_CHECK();
    int rc = reduce_theta(w, nb, a->theta, st);
    if (rc) return rc;
    // p_w^0 = PW(r^0, rho^0): momentum part only, no probe term
    if (nw > 0) {
        hipLaunchKernelGGL((k_wall_bwd<T, D>), dim3(grid_for(nw)), dim3(kBlock), 0, st, P, Q,
                           fmask(f->nbr_wf, f->cnt_wf, nw), nf, nw,
                           b->wkey, b->wpid, (const T*)b->woff, (const T*)b->nrm, (const T*)f->pw, f->pid,
                           (const T*)f->off, f->fstart, (const T*)f->vh, (const T*)f->rho,
                           (const T*)f->rho, (const double*)w.abar, (const double*)nullptr,
                           (const int32_t*)nullptr, 0, w.lam);
        SPH_LAUNCH_CHECK();
        hipLaunchKernelGGL((k_pw_bwd<T, D>), dim3(nb), dim3(kBlock), 0, st, P, Q,
                           fmask(f->nbr_fw, f->cnt_fw, nf), nf, nw, f->key, f->pid,
                           (const T*)f->off, (const T*)f->rho, (const T*)b->woff, b->wstart,
                           (const T*)f->pw, w.lam, a->xb, a->rhob, w.part);
        SPH_LAUNCH_CHECK();
        rc = reduce_theta(w, nb, a->theta, st);
        if (rc) return rc;
    }
    hipLaunchKernelGGL((k_init_theta<T, D>), dim3(nb), dim3(kBlock), 0, st, P, Q, make_grid(d), H, nf,
                       f->key, f->pid, (const T*)f->off, a->xb, a->rhob, w.part);
    SPH_LAUNCH_CHECK();
    return reduce_theta(w, nb, a->theta, st);
}

#define SPH_DISPATCH(fn, ...)                                                                        \
    (d->precision == SPH_F32 ? (d->dim == 2 ? fn<float, 2>(__VA_ARGS__) : fn<float, 3>(__VA_ARGS__)) \
                             : (d->dim == 2 ? fn<double, 2>(__VA_ARGS__) : fn<double, 3>(__VA_ARGS__)))

#define SPH_ADJ_CHECKS()                       \
    int rc_ = check_desc(d);                   \
    if (rc_) return rc_;                       \
    rc_ = check_buf(d, b);                     \
    if (rc_) return rc_;                       \
    rc_ = check_adj(d, b, a);                  \
    if (rc_) return rc_;                       \
    hipStream_t st = (hipStream_t)stream;

}  // namespace

extern "C" {

size_t sph_adjoint_work_bytes(const sph_desc* d, int64_t n_fluid, int64_t n_wall) {
    if (!d || n_fluid < 0 || n_wall < 0 || n_fluid > max_particles(d) || n_wall > max_particles(d)) return 0;
    return adj_layout(d, n_fluid, n_wall, nullptr).bytes;
}

int sph_adjoint_zero(const sph_desc* d, const sph_buffers* b, sph_adjoint* a, void* stream) {
    SPH_ADJ_CHECKS();
    const int64_t nf = b->n_fluid;
    const int64_t nd = (int64_t)d->dim * nf;
    double* arr[4] = {a->xb, a->vb, a->ab, a->rhob};
    const int64_t len[4] = {nd, nd, nd, nf};
    for (int k = 0; k < 4; ++k)
        if (len[k] > 0) {
            hipLaunchKernelGGL(k_zero_f64, dim3(grid_for(len[k])), dim3(kBlock), 0, st, arr[k], len[k]);
            SPH_LAUNCH_CHECK();
        }
    hipLaunchKernelGGL(k_zero_f64, dim3(1), dim3(kBlock), 0, st, a->theta, (int64_t)SPH_NTHETA);
    SPH_LAUNCH_CHECK();
    return SPH_OK;
}

int sph_forces_bwd(const sph_desc* d, const sph_buffers* b, const sph_frame* f, sph_adjoint* a,
                   void* stream) {
    SPH_ADJ_CHECKS();
    if ((rc_ = check_frame(b, f, false, true))) return rc_;
    return SPH_DISPATCH(forces_bwd_t, d, b, f, a, st);
}

int sph_wall_bc_bwd(const sph_desc* d, const sph_buffers* b, const sph_frame* f, sph_adjoint* a,
                    void* stream) {
    SPH_ADJ_CHECKS();
    if ((rc_ = check_frame(b, f, false, true))) return rc_;
    return SPH_DISPATCH(wall_bc_bwd_t, d, b, f, a, st);
}

int sph_density_bwd(const sph_desc* d, const sph_buffers* b, const sph_frame* f, sph_adjoint* a,
                    void* stream) {
    SPH_ADJ_CHECKS();
    if ((rc_ = check_frame(b, f, true, false))) return rc_;
    return SPH_DISPATCH(density_bwd_t, d, b, f, a, st);
}

int sph_step_bwd(const sph_desc* d, const sph_buffers* b, const sph_frame* cur, const sph_frame* next,
                 sph_adjoint* a, void* stream) {
    int rc = sph_forces_bwd(d, b, next, a, stream);
    if (!rc) rc = sph_wall_bc_bwd(d, b, next, a, stream);
    if (!rc) rc = sph_density_bwd(d, b, cur, a, stream);
    return rc;
}

int sph_init_bwd(const sph_desc* d, const sph_buffers* b, const sph_frame* f0, double H, sph_adjoint* a,
                 void* stream) {
    SPH_ADJ_CHECKS();
    if (!(H > 0.0)) return SPH_ERR_ARG;
    if (!f0 || (b->n_fluid > 0 && (!f0->key || !f0->pid || !f0->off || !f0->fstart || !f0->rho || !f0->vh)))
        return SPH_ERR_ARG;
    if (b->n_wall > 0 && !f0->pw) return SPH_ERR_ARG;
    return SPH_DISPATCH(init_bwd_t, d, b, f0, H, a, st);
}

}  // extern "C"
