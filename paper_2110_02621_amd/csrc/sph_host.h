// sph_host.h -- host-side helpers shared by the forward and adjoint
// translation units: run constants, grid, scratch layout, argument checks.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>

#include "sph.h"
#include "sph_device.h"

namespace sph {

constexpr int kScanThreads = 1024;
constexpr int kScanPer = 4;
constexpr int kScanTile = kScanThreads * kScanPer;
constexpr int kDiagVals = 8;  // M, P0, P1, P2, Ek, Ep, vmax, nonfinite

inline int grid_for(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

struct GridD {
    double lo[3];
    double L;
    int n[3];
    double X[3], V[3];  // tank position and velocity in the fixed frame (moving tank; else 0)
};

// Prescribed tank motion X(t) = A0 sin(2 pi f t) at t = step dt, with its
// velocity and acceleration (all 0 for a fixed tank).
struct Motion {
    double X[3], V[3], A[3];
};

inline bool moving(const sph_desc* d) { return d->motion_freq != 0.0; }

inline Motion motion_at(const sph_desc* d, int64_t step) {
    Motion m;
    const double w = 2.0 * M_PI * d->motion_freq, t = (double)step * d->dt;
    const double s = std::sin(w * t), c = std::cos(w * t);
    for (int k = 0; k < 3; ++k) {
        const double a = moving(d) && k < d->dim ? d->motion_amp[k] : 0.0;
        m.X[k] = a * s;
        m.V[k] = a * w * c;
        m.A[k] = -a * w * w * s;
    }
    return m;
}

// Tank velocity over the drift of step n: (X(t_{n+1}) - X(t_n)) / dt.
inline void drift_velocity(const sph_desc* d, int64_t n, double Vh[3]) {
    const Motion a = motion_at(d, n), b = motion_at(d, n + 1);
    for (int k = 0; k < 3; ++k) Vh[k] = (b.X[k] - a.X[k]) / d->dt;
}

template <typename T>
inline Par<T> make_par(const sph_desc* d) {
    Par<T> P;
    std::memset(&P, 0, sizeof(P));
    const double h = d->h;
    const double alpha = d->dim == 2 ? 7.0 / (4.0 * M_PI * h * h) : 21.0 / (16.0 * M_PI * h * h * h);
    const double vol = d->dim == 2 ? d->dx * d->dx : d->dx * d->dx * d->dx;
    P.nx = d->grid[0];
    P.ny = d->grid[1];
    P.nz = d->grid[2];
    P.penalty = d->penalty_all ? 1 : 0;
    P.L = T(d->cell);
    P.rc2 = T(4.0 * h * h);
    P.hinv = T(1.0 / h);
    P.alpha = T(alpha);
    P.gfac = T(-5.0 * alpha / (h * h));
    P.m = T(d->rho0 * vol);
    P.vol = T(vol);
    P.rho0 = T(d->rho0);
    P.c = T(d->c0);
    P.c2 = T(d->c0 * d->c0);
    P.cinv = T(1.0 / d->c0);
    P.inv_c2 = T(1.0 / (d->c0 * d->c0));
    P.mu2 = T(2.0 * d->mu);
    P.eta2 = T(0.01 * h * h);
    P.gamma_p = T(d->gamma_p);
    P.two_over_dx = T(2.0 / d->dx);
    for (int k = 0; k < 3; ++k) {
        P.g[k] = T(d->g[k]);
        P.gw[k] = T(d->g[k] - d->a_wall[k]);
    }
    P.dt = T(d->dt);
    P.half_dt = T(0.5 * d->dt);
    P.sigma0 = T(d->sigma0);
    P.rho0_over_sigma0 = T(d->rho0 / d->sigma0);
    P.psi_min = T(1e-4 / h);
    P.two_phase = d->two_phase ? 1 : 0;
    P.n_heavy = d->two_phase ? (int)d->n_heavy : 0;
    P.cross_phase = d->two_phase ? d->cross_phase : 0;
    P.rho0L = T(d->two_phase ? d->rho0_light : d->rho0);
    P.rho0L_over_sigma0 = T((d->two_phase ? d->rho0_light : d->rho0) / d->sigma0);
    return P;
}

inline GridD make_grid(const sph_desc* d) {
    GridD G;
    for (int k = 0; k < 3; ++k) {
        G.lo[k] = k < d->dim ? d->lo[k] : 0.0;
        G.n[k] = d->grid[k];
    }
    G.L = d->cell;
    for (int k = 0; k < 3; ++k) G.X[k] = G.V[k] = 0.0;
    return G;
}

// Grid with the tank's position and velocity at t = step dt.
inline GridD make_grid_at(const sph_desc* d, int64_t step) {
    GridD G = make_grid(d);
    const Motion m = motion_at(d, step);
    for (int k = 0; k < 3; ++k) {
        G.X[k] = m.X[k];
        G.V[k] = m.V[k];
    }
    return G;
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Neighbour masks of the current sorted state (see sph_buffers); {null}
// when absent.
inline NbrMask mask_ff(const sph_buffers* b) {
    return b->nbr_ff ? NbrMask{b->nbr_ff, b->cnt_ff, b->n_fluid} : NbrMask{nullptr, nullptr, 0};
}
inline NbrMask mask_fw(const sph_buffers* b) {
    return b->nbr_fw ? NbrMask{b->nbr_fw, b->cnt_fw, b->n_fluid} : NbrMask{nullptr, nullptr, 0};
}
inline NbrMask mask_wf(const sph_buffers* b) {
    return b->nbr_wf ? NbrMask{b->nbr_wf, b->cnt_wf, b->n_wall} : NbrMask{nullptr, nullptr, 0};
}

struct Scratch {
    int32_t* count;   // n_cells
    int32_t* slot;    // max(nf, nw)
    int32_t* perm;    // max(nf, nw)
    int32_t* tiles;   // scan tile sums
    int32_t* winv;    // n_wall: sorted index of each wall id (kept between calls)
    int32_t* wkey0;   // n_wall, unsorted wall keys (init only)
    void* woff0;      // dim * n_wall T, unsorted wall offsets (init only)
    double* part;     // diag partials
    void* sig;        // n_fluid T: sigma summed by the last momentum sweep
    // packed copies of the sorted state that the sweeps gather from
    // (Rec<T> = 4 T): pk[s] = (offset, rho[s] - rho0), vk[s] = (vel[s],
    // the particle's reference density) mirror the two density and
    // velocity copies; wk = (wall offset, p_w), nk = (wall normal, 0)
    void* pk[2];
    void* vk[2];
    void* wk;
    void* nk;
    uint8_t* wnear;  // n_cells: 1 when a wall particle lies in the cell's neighbour cells (set by sph_init)
    void* pd;        // n_fluid T: two phases, cross_phase 2: each heavy particle's dummy pressure
    size_t bytes;
};

inline Scratch layout(const sph_desc* d, int64_t nf, int64_t nw, void* base) {
    const size_t ts = d->precision == SPH_F64 ? 8 : 4;
    const int64_t nmax = nf > nw ? nf : nw;
    const int64_t ntiles = (d->n_cells + kScanTile - 1) / kScanTile + 1;
    const int64_t ndiag = (nf + kBlock - 1) / kBlock + 1;
    size_t o = 0;
    Scratch s;
    char* b = (char*)base;
    auto take = [&](size_t bytes) {
        char* p = b ? b + o : nullptr;
        o += align256(bytes > 0 ? bytes : 1);
        return (void*)p;
    };
    s.count = (int32_t*)take(sizeof(int32_t) * (size_t)(d->n_cells + 1));
    s.slot = (int32_t*)take(sizeof(int32_t) * (size_t)nmax);
    s.perm = (int32_t*)take(sizeof(int32_t) * (size_t)nmax);
    s.tiles = (int32_t*)take(sizeof(int32_t) * (size_t)ntiles);
    s.winv = (int32_t*)take(sizeof(int32_t) * (size_t)nw);
    s.wkey0 = (int32_t*)take(sizeof(int32_t) * (size_t)nw);
    s.woff0 = take(ts * (size_t)d->dim * (size_t)nw);
    s.part = (double*)take(sizeof(double) * kDiagVals * (size_t)ndiag);
    s.sig = take(ts * (size_t)nf);
    for (int k = 0; k < 2; ++k) s.pk[k] = take(4 * ts * (size_t)nf);
    for (int k = 0; k < 2; ++k) s.vk[k] = take(4 * ts * (size_t)nf);
    s.wk = take(4 * ts * (size_t)nw);
    s.nk = take(4 * ts * (size_t)nw);
    s.wnear = (uint8_t*)take((size_t)d->n_cells);
    s.pd = take(d->two_phase && d->cross_phase == 2 ? ts * (size_t)nf : 0);
    s.bytes = o;
    return s;
}

#define SPH_LAUNCH_CHECK()                                 \
    do {                                                   \
        if (hipGetLastError() != hipSuccess) return SPH_ERR_LAUNCH; \
    } while (0)

inline int check_desc(const sph_desc* d) {
    if (!d) return SPH_ERR_ARG;
    if (d->dim != 2 && d->dim != 3) return SPH_ERR_CONFIG;
    if (d->precision != SPH_F32 && d->precision != SPH_F64) return SPH_ERR_CONFIG;
    if (!(d->cell > 0.0) || d->n_cells <= 0) return SPH_ERR_CONFIG;
    return SPH_OK;
}

// Largest particle count of either set.  Every gather forms a 32-bit byte
// offset from its array's base (ldg, ld4), so a record array stays below
// 4 GiB: 2^28 - 1 particles in FP32 (16-byte records), 2^27 - 1 in FP64.
inline int64_t max_particles(const sph_desc* d) {
    return d->precision == SPH_F32 ? (int64_t{1} << 28) - 1 : (int64_t{1} << 27) - 1;
}

// Every buffer of the state and the outputs, scratch aside.
inline int check_state(const sph_desc* d, const sph_buffers* b) {
    if (!b) return SPH_ERR_ARG;
    if (b->n_fluid < 0 || b->n_wall < 0) return SPH_ERR_ARG;
    if (b->n_fluid > max_particles(d) || b->n_wall > max_particles(d)) return SPH_ERR_ARG;
    if (b->sel_vel < 0 || b->sel_vel > 1 || b->sel_rho < 0 || b->sel_rho > 1) return SPH_ERR_ARG;
    if (!b->status || !b->diag || !b->fstart || !b->wstart) return SPH_ERR_ARG;
    if (b->n_fluid > 0) {
        for (int c = 0; c < 2; ++c)
            if (!b->key[c] || !b->pid[c] || !b->off[c] || !b->vel[c] || !b->rho[c]) return SPH_ERR_ARG;
        if (!b->acc) return SPH_ERR_ARG;
    }
    if (b->n_wall > 0 && (!b->wkey || !b->wpid || !b->woff || !b->pw || !b->nrm)) return SPH_ERR_ARG;
    if (b->n_probe < 0 || (b->n_probe > 0 && !b->probe)) return SPH_ERR_ARG;
    const bool masks = b->nbr_ff || b->nbr_fw || b->nbr_wf;
    if (masks) {  // all three or none
        if (!b->nbr_ff || !b->nbr_fw || !b->nbr_wf || !b->cnt_ff || !b->cnt_fw || !b->cnt_wf) return SPH_ERR_ARG;
    }
    return SPH_OK;
}

inline int check_buf(const sph_desc* d, const sph_buffers* b) {
    const int rc = check_state(d, b);
    if (rc) return rc;
    if (!b->scratch || b->scratch_bytes < sph_scratch_bytes(d, b->n_fluid, b->n_wall)) return SPH_ERR_ARG;
    if (((uintptr_t)b->scratch & 255) != 0) return SPH_ERR_ARG;
    return SPH_OK;
}


}  // namespace sph
