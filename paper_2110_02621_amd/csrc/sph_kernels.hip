// sph_kernels.hip -- gfx950 kernels of the SPH hot path and the C ABI of
// include/sph.h.  One source, instantiated for T = float and T = double and
// for 2-D and 3-D.
//
// Method: Rezavand, Zhang & Hu (arXiv 2110.02621).  Readings of points the
// paper leaves open (the same as the FP64 oracle's):
//   - kernel: quintic Wendland C2, kappa = 2 (Sec. 2.3, Sec. 4);
//   - Eq. (12) with the fluid density in the hydrostatic term, p_w = 0
//     without fluid neighbours; wall density from the EOS and wall mass
//     rho0 dx^d;
//   - Eq. (17) at the start of each step with rho* = current density and a
//     scalar sigma^0 (full lattice sum);
//   - viscous term of Morris, Fox & Zhu (1997) with no-slip walls;
//   - penalty, Eqs. (13)-(15): delta = 2 |(r_i - r_w) . n_w| / dx and
//     F_p = -2 gamma_p sum m/(rho_i rho_w) (1 - delta)^2 |p_i e . n_w| W' n_w;
//   - normals, Eq. (16): n_w = 0 when |Psi| h <= 1e-4.
//
// Data layout (structure of arrays, sorted by cell): fluid key/pid int32,
// offsets, velocities, accelerations T[dim][n], density as rho - rho0 in T.
// Positions are cell + offset so that pair distances keep full relative
// precision in FP32 regardless of the tank size.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <type_traits>

#include "sph.h"
#include "sph_device.h"
#include "sph_host.h"

using namespace sph;

namespace {

// ---------------------------------------------------------------------------
// Small helpers
// ---------------------------------------------------------------------------


__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_f64(double* __restrict__ p, int64_t n, double v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// Counting sort by cell key (the sorting part of the neighbour search, Sec. 3, Table 1).
//   1. histogram: slot_i = atomic fetch-add on count[key_i] (the count per
//      cell is exact; the slot order inside a cell is arbitrary);
//   2. exclusive scan of the counts -> cell start table;
//   3. place: perm[start[key_i] + slot_i] = i;
//   4. rank of each entry among its cell's entries: for the fluid by x
//      offset, ties by source index, for the walls by source index (their
//      prior order); deterministic either way;
//   5. gather of every field through perm.
// ---------------------------------------------------------------------------

// The keys arrive nearly sorted (the previous order, drifted by less than
// a cell), so runs of equal keys are common inside a wave: each run's first
// lane adds the run length with one atomic and the run takes consecutive
// slots after the returned base.
__global__ void __launch_bounds__(kBlock) k_hist(const int32_t* __restrict__ key, int64_t n,
                                                  int32_t* __restrict__ count,
                                                  int32_t* __restrict__ slot) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < n;
    const int k = valid ? key[i] : -1;
    const int lane = threadIdx.x & 63;
    const int prev = __shfl_up(k, 1, 64);
    const bool head = valid && (lane == 0 || prev != k);
    const uint64_t heads = __ballot(head);
    const uint64_t vmask = __ballot(valid);
    // this lane's run: from the last head at or below it to the next head
    const uint64_t below = heads & ((lane == 63) ? ~0ull : ((2ull << lane) - 1));
    const int first = 63 - __builtin_clzll(below | 1ull);
    const uint64_t above = heads & ~((2ull << lane) - 1) & ((lane == 63) ? 0ull : ~0ull);
    const int next = above ? __builtin_ctzll(above) : 64;
    const int vend = 64 - __builtin_clzll(vmask | 1ull);  // one past the last valid lane
    const int len = min(next, vend) - first;
    int base = 0;
    if (head) base = atomicAdd(&count[k], len);
    base = __shfl(base, first, 64);
    if (valid) slot[i] = base + (lane - first);
}


// Exclusive scan of one value per thread over a block of kScanThreads.
__device__ __forceinline__ int block_exclusive_scan(int v, int* waves, int& total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) waves[wid] = x;
    __syncthreads();
    if (wid == 0) {
        const int nw = kScanThreads / 64;
        int w = lane < nw ? waves[lane] : 0;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(w, o, 64);
            if (lane >= o) w += y;
        }
        if (lane < nw) waves[lane] = w;
    }
    __syncthreads();
    const int base = wid > 0 ? waves[wid - 1] : 0;
    total = waves[kScanThreads / 64 - 1];
    __syncthreads();
    return base + x - v;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(const int32_t* __restrict__ cnt,
                                                               int64_t n,
                                                               int32_t* __restrict__ tile_sum) {
    __shared__ int waves[kScanThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) s += base + k < n ? cnt[base + k] : 0;
    int total;
    block_exclusive_scan(s, waves, total);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

// Single block: exclusive scan of the tile sums in place.
__global__ void __launch_bounds__(kScanThreads) k_scan_tiles(int32_t* __restrict__ tile_sum,
                                                              int ntiles) {
    __shared__ int waves[kScanThreads / 64];
    int carry = 0;
    for (int b = 0; b < ntiles; b += kScanThreads) {
        const int i = b + threadIdx.x;
        const int v = i < ntiles ? tile_sum[i] : 0;
        int total;
        const int e = block_exclusive_scan(v, waves, total);
        if (i < ntiles) tile_sum[i] = carry + e;
        carry += total;
    }
}

__global__ void __launch_bounds__(kScanThreads) k_scan_down(const int32_t* __restrict__ cnt,
                                                             int64_t n,
                                                             const int32_t* __restrict__ tile_off,
                                                             int32_t* __restrict__ start,
                                                             int32_t n_total) {
    __shared__ int waves[kScanThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    int v[kScanPer];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        v[k] = base + k < n ? cnt[base + k] : 0;
        s += v[k];
    }
    int total;
    int e = block_exclusive_scan(s, waves, total) + tile_off[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        if (base + k < n) start[base + k] = e;
        e += v[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) start[n] = n_total;
}

__global__ void __launch_bounds__(kBlock) k_place(const int32_t* __restrict__ key,
                                                   const int32_t* __restrict__ slot, int64_t n,
                                                   const int32_t* __restrict__ start,
                                                   int32_t* __restrict__ perm) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) perm[start[key[i]] + slot[i]] = (int32_t)i;
}

// In-cell order: each entry's rank among the entries of its cell by x
// offset (ox), ties by source index, or by source index alone without ox;
// either is a strict total order, so the permutation is the same whatever
// order the histogram atomics handed out slots in.  The fluid is ordered by
// x (the pair sweeps run faster on that order: the lanes of a cell then
// find their neighbours at nearby record indices); the walls keep their
// source order.  One thread per entry; the cell's few entries are read from
// cache.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_cellrank(const int32_t* __restrict__ key,
                                                      const int32_t* __restrict__ start,
                                                      const int32_t* __restrict__ placed, int64_t n,
                                                      const T* __restrict__ ox, int32_t* __restrict__ perm) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int v = placed[p];
    const int c = key[v];
    const int a = start[c], b = start[c + 1];
    int r = 0;
    if (ox) {
        const T xv = ox[v];
        auto before = [&](int u, T xu) { return (xu < xv || (xu == xv && u < v)) ? 1 : 0; };
        int q = a;
        for (; q + 4 <= b; q += 4) {  // four independent index-then-offset loads in flight
            const int u0 = placed[q], u1 = placed[q + 1], u2 = placed[q + 2], u3 = placed[q + 3];
            const T x0 = ox[u0], x1 = ox[u1], x2 = ox[u2], x3 = ox[u3];
            r += before(u0, x0) + before(u1, x1) + before(u2, x2) + before(u3, x3);
        }
        for (; q < b; ++q) {
            const int u = placed[q];
            r += before(u, ox[u]);
        }
    } else {
        for (int q = a; q < b; ++q) r += placed[q] < v ? 1 : 0;
    }
    perm[a + r] = v;
}

template <typename T, int D>
__global__ void __launch_bounds__(kBlock)
    k_gather_fluid(Par<T> P, const int32_t* __restrict__ perm, int64_t n, const int32_t* __restrict__ key_in,
                   const int32_t* __restrict__ pid_in, const T* __restrict__ off_in,
                   const T* __restrict__ vel_in, const T* __restrict__ rho_in,
                   int32_t* __restrict__ key_out, int32_t* __restrict__ pid_out,
                   T* __restrict__ off_out, T* __restrict__ vel_out, T* __restrict__ rho_out,
                   Rec<T>* __restrict__ pk_out, Rec<T>* __restrict__ vk_out) {
    const int64_t i = global_index<kChunk>();
    if (i >= n) return;
    const int64_t s = perm[i];
    key_out[i] = key_in[s];
    const int32_t id = pid_in[s];
    pid_out[i] = id;
    const T r = rho_in[s];
    rho_out[i] = r;
    T o[3] = {0, 0, 0}, v[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < D; ++k) {
        o[k] = off_in[k * n + s];
        v[k] = vel_in[k * n + s];
        off_out[k * n + i] = o[k];
        vel_out[k * n + i] = v[k];
    }
    pk_out[i] = Rec<T>{o[0], o[1], o[2], r};
    vk_out[i] = Rec<T>{v[0], v[1], v[2], ref_density(P, id)};
}

template <typename T, int D>
__global__ void __launch_bounds__(kBlock)
    k_gather_wall(const int32_t* __restrict__ perm, int64_t n, const int32_t* __restrict__ key_in,
                  const T* __restrict__ off_in, int32_t* __restrict__ key_out,
                  int32_t* __restrict__ pid_out, T* __restrict__ off_out,
                  int32_t* __restrict__ inv) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t s = perm[i];
    key_out[i] = key_in[s];
    pid_out[i] = s;
    inv[s] = (int32_t)i;
#pragma unroll
    for (int k = 0; k < D; ++k) off_out[k * n + i] = off_in[k * n + s];
}

// Packed wall records: offset with p_w (w filled by the wall pressure) and
// the normal.
template <typename T, int D>
__global__ void __launch_bounds__(kBlock)
    k_pack_walls(int64_t nw, const T* __restrict__ woff, const T* __restrict__ nrm,
                 Rec<T>* __restrict__ wk, Rec<T>* __restrict__ nk) {
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= nw) return;
    wk[w] = Rec<T>{woff[w], woff[nw + w], D == 3 ? woff[2 * nw + w] : T(0), T(0)};
    nk[w] = Rec<T>{nrm[w], nrm[nw + w], D == 3 ? nrm[2 * nw + w] : T(0), T(0)};
}

// Cells with at least one wall particle among their 27 (3-D) or 9 (2-D)
// neighbour cells (the walls are sorted once, so this is built once).
template <typename T, int D>
__global__ void __launch_bounds__(kBlock)
    k_wall_near(Par<T> P, int64_t n_cells, const int32_t* __restrict__ wstart, uint8_t* __restrict__ near) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_cells) return;
    int c[3];
    cell_of(P, (int)k, c);
    const int x0 = max(c[0] - 1, 0), x1 = min(c[0] + 1, P.nx - 1);
    bool any = false;
    for (int dz = (D == 3 ? -1 : 0); dz <= (D == 3 ? 1 : 0); ++dz)
        for (int dy = -1; dy <= 1; ++dy) {
            const int y = c[1] + dy, z = c[2] + dz;
            if (y < 0 || y >= P.ny || z < 0 || z >= (D == 3 ? P.nz : 1)) continue;
            const int row = P.nx * (y + P.ny * z);
            any = any || wstart[row + x1 + 1] > wstart[row + x0];
        }
    near[k] = any ? 1 : 0;
}

// ---------------------------------------------------------------------------
// Position conversion: absolute double -> cell + offset in T.
// ---------------------------------------------------------------------------

template <typename T, int D>
__global__ void __launch_bounds__(kBlock)
    k_to_cells(const double* __restrict__ pos, int64_t n, GridD G, int32_t* __restrict__ key,
               T* __restrict__ off, uint32_t* __restrict__ status) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const T L = T(G.L);
    int c[3] = {0, 0, 0};
    bool outside = false;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const double x = (pos[k * n + i] - G.X[k]) - G.lo[k];
        double f = floor(x / G.L);
        int ck = (int)fmax(fmin(f, (double)(G.n[k] - 1)), 0.0);
        if (!(f >= 0.0 && f <= (double)(G.n[k] - 1))) outside = true;
        T o = T(x - (double)ck * G.L);
        if (o < T(0)) o = T(0);
        if (o >= L) {  // rounding up to L: same point as offset 0 of the next cell
            if (ck + 1 < G.n[k]) {
                ++ck;
                o = T(0);
            } else {
                o = L * T(0.9999999);
                outside = true;
            }
        }
        c[k] = ck;
        off[k * n + i] = o;
    }
    if (outside) atomicAdd(&status[SPH_STATUS_OUT_OF_GRID], 1u);
    key[i] = c[0] + G.n[0] * (c[1] + G.n[1] * c[2]);
}

// Initial velocity and density into the current copies (pid = input index).
template <typename T, int D>
__global__ void __launch_bounds__(kBlock)
    k_init_state(Par<T> P, GridD G, int64_t n, const double* __restrict__ vel,
                 const double* __restrict__ rho, int32_t* __restrict__ pid, T* __restrict__ vel_out,
                 T* __restrict__ drho_out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    pid[i] = (int32_t)i;
    for (int k = 0; k < D; ++k) vel_out[k * n + i] = T(vel[k * n + i] - G.V[k]);
    drho_out[i] = T(rho[i] - (double)ref_density(P, (int)i));
}

// ---------------------------------------------------------------------------
// Wall normals, Eq. (16): Psi_w = -sum_{j in walls} dx^d grad_w W_wj.
// ---------------------------------------------------------------------------

template <typename T, int D>
__global__ void __launch_bounds__(kBlock)
    k_normals(Par<T> P, int64_t nw, const int32_t* __restrict__ wkey, const T* __restrict__ woff,
              const int32_t* __restrict__ wstart, T* __restrict__ nrm) {
    const int64_t w = global_index<kChunk>();
    if (w >= nw) return;
    const T* o0 = woff;
    const T* o1 = woff + nw;
    const T* o2 = woff + 2 * nw;
    int c[3];
    cell_of(P, wkey[w], c);
    const T oi[3] = {o0[w], o1[w], D == 3 ? o2[w] : T(0)};
    T psi[3] = {0, 0, 0};
    for_neighbours<T, D>(P, wstart, o0, o1, o2, c, oi, [&](int, const T d[3], T r2, uint32_t) {
        if (r2 > T(0)) {
            const T F = wendland_F(P, root(r2));
#pragma unroll
            for (int k = 0; k < D; ++k) psi[k] -= P.vol * F * d[k];
        }
    });
    T n2 = T(0);
#pragma unroll
    for (int k = 0; k < D; ++k) n2 += psi[k] * psi[k];
    const T nn = root(n2);
    const bool zero = !(nn > P.psi_min);
#pragma unroll
    for (int k = 0; k < D; ++k) nrm[k * nw + w] = zero ? T(0) : psi[k] / nn;
}

// ---------------------------------------------------------------------------
// Density update: sigma_i, Eq. (17) reinitialisation, half kick Eq. (19),
// drift Eq. (20) with cell renormalisation.
// ---------------------------------------------------------------------------

// Records per wave staged in LDS for one stencil row (a row of a wave that
// spans about four cells holds ~100 particles; longer rows are gathered).
// A block staging for all its waves at once has kWaves * kStage records,
// enough for a row and its mirror image of a block in one row of cells
// (~2 x 290 on a full lattice).  The continuity sweep needs fewer registers
// and stages fewer records (more pairs of rows go one row at a time), which
// fits a seventh block per CU and is faster; the mask builder stages
// position records only, and more of them.
constexpr int kStage = 192;   // momentum: 2 x 768 records per block, 6 blocks (80 VGPRs)
constexpr int kStageC = 160;  // continuity: 2 x 640 records per block, 7 blocks
constexpr int kStageM = 256;  // mask builder: 256 position records per wave
constexpr int kWaves = kBlock / 64;

// The fluid-fluid part of a pair sweep for particle i: block-staged when the
// block lies in one row of cells (threads regrouped, see regroup_block),
// else wave-staged when the wave does, else gathered from memory; lanes
// whose masks overflowed walk the cells.  fluid(j, d, r2, code, q, u) takes
// the position record q and velocity record u of j; fluid_g(j, d, r2, code,
// q) the same with u loaded from memory.
template <int STAGE, typename T, int D, typename F, typename G>
__device__ __forceinline__ void fluid_sweep(const Par<T>& P, const NbrMask& LF, const int32_t* __restrict__ fstart,
                                            const Rec<T>* __restrict__ pk, const Rec<T>* __restrict__ vk,
                                            const int32_t* __restrict__ key, Rec<T>* stage, bool block_mode,
                                            const WaveSpan& SB, bool act, int64_t ib, int64_t nf, int64_t i,
                                            const int c[3], const T oi[3], F&& fluid, G&& fluid_g) {
    if (block_mode) {
        const bool m = act && LF.count[i] >= 0;
        mask_block<T, D, kWaves * STAGE>(P, fstart, pk, vk, (SPH_LDS Rec<T>*)stage,
                                         (SPH_LDS Rec<T>*)(stage + kWaves * STAGE), SB, m, c, oi, LF.mask,
                                          LF.n, i, fluid);
        if (act && !m) walk_src<T, D>(P, fstart, PackSrc<T>{pk}, c, oi, fluid_g);
        return;
    }
    const WaveSpan S = wave_span(P, key, ib, nf);
    if (LF.mask && S.one_row) {
        const bool m = act && LF.count[i] >= 0;
        const int wv = threadIdx.x >> 6;
        mask_staged<T, D, STAGE>(P, fstart, pk, vk, (SPH_LDS Rec<T>*)(stage + wv * STAGE),
                                 (SPH_LDS Rec<T>*)(stage + (kWaves + wv) * STAGE), S, m, c, oi, LF.mask,
                                  LF.n, i, fluid);
        if (act && !m) walk_src<T, D>(P, fstart, PackSrc<T>{pk}, c, oi, fluid_g);
    } else if (act) {
        visit4<T, D>(P, LF, i, fstart, PackSrc<T>{pk}, c, oi, fluid_g);
    }
}

template <typename T>
__device__ __forceinline__ void kahan_add(T& s, T& comp, T v) {
#pragma clang fp contract(off)  // the same rounding wherever it is inlined
    if (std::is_same<T, float>::value) {
        const T y = v - comp;
        const T t = s + y;
        comp = (t - s) - y;
        s = t;
    } else {
        s += v;
    }
}

// Move an offset by dx and keep it in [0, L): returns the cell shift.
// One-cell moves are exact (Sterbenz); longer ones are counted.
template <typename T>
__device__ __forceinline__ int renormalise(T& o, T L, uint32_t* status) {
    if (o >= T(0) && o < L) return 0;
    if (o >= L && o < T(2) * L) {
        o = o - L;
        return 1;
    }
    if (o < T(0) && o >= -L) {
        const T t = o + L;
        if (t < L) {
            o = t;
            return -1;
        }
        o = T(0);  // o + L rounds to L: the point is the start of this cell
        return 0;
    }
    atomicAdd(&status[SPH_STATUS_FAST], 1u);
    if (!(o == o) || absv(o) > T(1e6) * L) {  // non-finite or absurd: park at the cell start
        o = T(0);
        return 0;
    }
    const T f = floorv(o / L);
    o = o - f * L;
    if (o < T(0)) o = T(0);
    if (o >= L) o = T(0);
    return (int)f;
}

template <typename T, int D>
__global__ void __launch_bounds__(kBlock)
    k_density(Par<T> P, NbrMask LF, NbrMask LW, int64_t nf, int64_t nw, const int32_t* __restrict__ key,
              const int32_t* __restrict__ pid, const T* __restrict__ off,
              const int32_t* __restrict__ fstart, const T* __restrict__ woff,
              const int32_t* __restrict__ wstart, T* __restrict__ vel, T* __restrict__ drho,
              const T* __restrict__ acc, int32_t* __restrict__ key_out,
              int32_t* __restrict__ pid_out, T* __restrict__ off_out, T* __restrict__ sigma_out,
              const T* __restrict__ sigma_in, Rec<T>* __restrict__ pk, Rec<T>* __restrict__ vk,
              uint32_t* __restrict__ status) {
    const int64_t i = global_index<kChunk>();
    if (i >= nf) return;
    const T* o0 = off;
    const T* o1 = off + nf;
    const T* o2 = off + 2 * nf;
    int c[3];
    cell_of(P, key[i], c);
    const T oi[3] = {o0[i], o1[i], D == 3 ? o2[i] : T(0)};
    T s = T(0), comp = T(0);
    if (sigma_in) {
        s = sigma_in[i];  // summed by the momentum sweep over the same pairs, in the same order
    } else {
        auto addW = [&](int, const T*, T r2, uint32_t) { kahan_add(s, comp, wendland_W(P, pair_r(r2))); };
        visit<T, D>(P, LF, i, fstart, o0, o1, o2, c, oi, addW);
        if (nw > 0 && (!LW.mask || LW.count[i] != 0))
            visit<T, D>(P, LW, i, wstart, woff, woff + nw, woff + 2 * nw, c, oi, addW);
    }
    if (sigma_out) sigma_out[i] = s;
    // Eq. (17) in deviations from rho0: rho_s - rho0 = rho0 (sigma - sigma0)/sigma0.
    const int id = pid[i];
    const bool light = P.two_phase && id >= P.n_heavy;
    T dtil;
    if (light) {
        // Eq. (18), internal flow: rho - rho0_light = rho0_light (sigma - sigma0)/sigma0
        dtil = P.rho0L_over_sigma0 * (s - P.sigma0);
    } else {
        const T drs = P.rho0_over_sigma0 * (s - P.sigma0);
        const T dstar = drho[i];
        const T excess = dstar - drs;
        dtil = excess > T(0) ? drs + excess * P.rho0 / (P.rho0 + dstar) : drs;
    }
    drho[i] = dtil;
    // Eqs. (19)-(20): half kick, drift, renormalise the cell.
    int cn[3] = {c[0], c[1], c[2]};
    const int nmax[3] = {P.nx, P.ny, P.nz};
    bool out = false;
    T vh[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const T v = vel[k * nf + i] + P.half_dt * acc[k * nf + i] + P.fk[k];
        vel[k * nf + i] = v;
        vh[k] = v;
        T o = oi[k] + P.dt * v;
        int ck = c[k] + renormalise(o, P.L, status);
        if (ck < 0) {
            ck = 0;
            o = T(0);
            out = true;
        } else if (ck >= nmax[k]) {
            ck = nmax[k] - 1;
            o = P.L * T(0.9999999);
            out = true;
        }
        cn[k] = ck;
        off_out[k * nf + i] = o;
    }
    if (out) atomicAdd(&status[SPH_STATUS_OUT_OF_GRID], 1u);
    key_out[i] = cn[0] + P.nx * (cn[1] + P.ny * cn[2]);
    pid_out[i] = id;
    // packed copies of the sorted state: same offsets, the new density and velocity
    pk[i] = Rec<T>{oi[0], oi[1], oi[2], dtil};
    vk[i] = Rec<T>{vh[0], vh[1], vh[2], light ? P.rho0L : P.rho0};
}

// ---------------------------------------------------------------------------
// Wall pressure, Eq. (12), one thread per wall particle.
// ---------------------------------------------------------------------------

template <typename T, int D, bool MP>
__global__ void __launch_bounds__(kBlock)
    k_wall_bc(Par<T> P, NbrMask LWF, int64_t nf, int64_t nw, const int32_t* __restrict__ wkey,
              const int32_t* __restrict__ fstart, const Rec<T>* __restrict__ pk,
              const Rec<T>* __restrict__ vk, Rec<T>* __restrict__ wk, T* __restrict__ pw) {
    const int64_t w = global_index<kChunk>();
    if (w >= nw) return;
    if (nf == 0 || (LWF.mask && LWF.count[w] == 0)) {  // no fluid neighbour: Eq. (12) gives 0
        pw[w] = T(0);
        wk[w].w = T(0);
        return;
    }
    int c[3];
    cell_of(P, wkey[w], c);
    const Rec<T> me = wk[w];
    const T ow[3] = {me.x, me.y, me.z};
    T sW = T(0), sP = T(0), sR[3] = {0, 0, 0};
    if (nf > 0)
        visit4<T, D>(P, LWF, w, fstart, PackSrc<T>{pk}, c, ow,
                             [&](int f, const T d[3], T r2, uint32_t, const Rec<T>& q) {
                                 const T W = wendland_W(P, root(r2));
                                 const T dr = q.w;
                                 if (MP) {
                                     // two phases: Eq. (12) divided by rho_f term by term
                                     const T rinv = T(1) / (ld4(vk, f).w + dr);
                                     sW += W * rinv;
                                     sP += P.c2 * dr * W * rinv;
#pragma unroll
                                     for (int k = 0; k < D; ++k) sR[k] += W * d[k];
                                 } else {
                                     sW += W;
                                     sP += P.c2 * dr * W;
                                     const T rW = (P.rho0 + dr) * W;
#pragma unroll
                                     for (int k = 0; k < D; ++k) sR[k] += rW * d[k];
                                 }
                             });
    T gR = T(0);
#pragma unroll
    for (int k = 0; k < D; ++k) gR += P.gw[k] * sR[k];
    const T p = sW > T(0) ? (sP + gR) / sW : T(0);
    pw[w] = p;
    wk[w].w = p;
}

// Probe integral: diag[PROBE] += dt * mean(p_w over the probe walls).
template <typename T>
__global__ void __launch_bounds__(kBlock)
    k_probe(const T* __restrict__ pw, const int32_t* __restrict__ inv, int64_t nw,
            const int32_t* __restrict__ probe, int np, double dt, double* __restrict__ diag) {
    __shared__ double red[kBlock];
    double s = 0.0;
    for (int a = threadIdx.x; a < np; a += kBlock) {
        const int32_t id = probe[a];
        if (id >= 0 && id < nw) s += (double)pw[inv[id]];  // ids outside the walls add 0
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) diag[SPH_DIAG_PROBE] += dt * red[0] / (double)np;
}

// ---------------------------------------------------------------------------
// Mass conservation, Eq. (9) with Eqs. (7)-(8), and Eq. (21).
// With v* = U* e + (rho_i v_i + rho_j v_j)/(rho_i + rho_j) - Ubar e one has
// (v_i - v*) . grad W = F [rho_j (v_ij . r_ij) + (p_i - p_j) r / c]/(rho_i + rho_j)
// with F = W'(r)/r, so per pair the sum gains
// F [rho_j (v_ij . r_ij) + (p_i - p_j) r / c] / (rho_j (rho_i + rho_j)).
// ---------------------------------------------------------------------------

template <typename T, int D, bool MP>
__global__ void __launch_bounds__(kBlock)
    k_continuity(Par<T> P, NbrMask LF, NbrMask LW, int64_t nf, int64_t nw, const int32_t* __restrict__ key,
                 const int32_t* __restrict__ pid, const int32_t* __restrict__ fstart, const Rec<T>* __restrict__ pk,
                 const Rec<T>* __restrict__ vk, const int32_t* __restrict__ wstart,
                 const Rec<T>* __restrict__ wk, T* __restrict__ drho_out, Rec<T>* __restrict__ pk_out) {
    __shared__ Rec<T> stage[2 * kWaves * kStageC];
    __shared__ int perm[kBlock];
    __shared__ int hist[16];
    const int64_t blk0 = (int64_t)logical_block() * kBlock;
    if (blk0 >= nf) return;  // the whole block is past the end
    const WaveSpan SB = span_of(P, key, blk0, (blk0 + kBlock < nf ? blk0 + kBlock : nf) - 1);
    const bool block_mode = LF.mask && SB.one_row;
    const int64_t i0 = block_mode ? regroup_block<T, D>(P, pk, blk0, nf, hist, perm) : blk0 + threadIdx.x;
    const int64_t ib = i0 - (threadIdx.x & 63);
    if (!block_mode && ib >= nf) return;  // the whole wave is past the end
    const bool act = i0 < nf;
    const int64_t i = act ? i0 : nf - 1;
    int c[3];
    cell_of(P, key[i], c);
    const Rec<T> me = pk[i];
    const Rec<T> mv = vk[i];
    const T oi[3] = {me.x, me.y, me.z};
    const T vi[3] = {mv.x, mv.y, mv.z};
    const T dri = me.w;
    const bool light = MP && pid[i] >= P.n_heavy;
    const T r0i = light ? P.rho0L : P.rho0;  // own reference density
    const T rho_i = r0i + dri;
    T sum = T(0);
    T sig = T(0), comp = T(0);  // two phases: sigma at these positions for the light phase
    auto fluid = [&](int, const T d[3], T r2, uint32_t, const Rec<T>& q, const Rec<T>& vj) {
        // no branch for r = 0 (the particle itself, or a coincident one):
        // every part of its term carries r or d, so it adds an exact zero,
        // and the velocity record is read without waiting on r2.  Two
        // phases sum sigma here too, in the form every sigma sum takes.
        const T r = MP ? pair_r(r2) : root(r2);
        const KernelWF<T> k = wendland_WF(P, r);
        if (MP) kahan_add(sig, comp, k.W);
        const T F = k.F;
        const T drj = q.w;
        const T r0j = MP ? vj.w : P.rho0;
        const T rho_j = r0j + drj;
        const T vjk[3] = {vj.x, vj.y, vj.z};
        T vd = T(0);
#pragma unroll
        for (int k = 0; k < D; ++k) vd += (vi[k] - vjk[k]) * d[k];
        const T qq = rcp(rho_j * (rho_i + rho_j));
        const T term = F * qq * (rho_j * vd + P.c * (dri - drj) * r);  // c^2 (rho_i - rho_j) r / c
        sum += MP ? r0j * term : term;  // m_j = rho0_j dx^d
    };
    auto fluid_g = [&](int j, const T d[3], T r2, uint32_t code, const Rec<T>& q) {
        fluid(j, d, r2, code, q, ld4(vk, j));
    };
    fluid_sweep<kStageC, T, D>(P, LF, fstart, pk, vk, key, stage, block_mode, SB, act, ib, nf, i, c, oi, fluid,
                               fluid_g);
    if (!act) return;
    if (nw > 0 && (!LW.mask || LW.count[i] != 0))  // no wall neighbour: nothing to add
        visit_walls<T, D>(P, LW, i, wstart, wk, nullptr, c, oi,
                     [&](int, const T d[3], T r2, const Rec<T>& q, const Rec<T>&) {
                         const T r = MP ? pair_r(r2) : root(r2);
                         const KernelWF<T> k = wendland_WF(P, r);
                         if (MP) kahan_add(sig, comp, k.W);
                         if (!(r2 > T(0))) return;
                         const T F = k.F;
                         const T p_w = q.w;
                         const T rho_w = r0i + p_w * P.inv_c2;  // the wall takes i's phase
                         T vd = T(0);
#pragma unroll
                         for (int k = 0; k < D; ++k) vd += vi[k] * d[k];
                         const T qq = rcp(rho_w * (rho_i + rho_w));
                         const T term = F * qq * (rho_w * vd + (P.c2 * dri - p_w) * r * P.cinv);
                         sum += MP ? r0i * term : term;
                     });
    T dnew = MP ? dri + P.dt * (T(2) * rho_i * P.vol * sum) : dri + P.dt * (T(2) * rho_i * P.m * sum);
    if (light) dnew = P.rho0L_over_sigma0 * (sig - P.sigma0);  // light phase: number density at r^{n+1}
    drho_out[i] = dnew;
    pk_out[i] = Rec<T>{me.x, me.y, me.z, dnew};
}

// ---------------------------------------------------------------------------
// Two phases, cross_phase 2: the pressure each heavy particle carries as a
// moving wall dummy of the light phase, extrapolated from its light
// neighbours by the two-phase form of Eq. (12) (each term divided by rho_f),
// with g - a_w of the tank; 0 for light particles and for heavy ones
// without light neighbours.
// ---------------------------------------------------------------------------

template <typename T, int D>
__global__ void __launch_bounds__(kBlock)
    k_dummy_pressure(Par<T> P, NbrMask LF, int64_t nf, const int32_t* __restrict__ key,
                     const int32_t* __restrict__ pid, const int32_t* __restrict__ fstart,
                     const Rec<T>* __restrict__ pk, const Rec<T>* __restrict__ vk, T* __restrict__ pd) {
    const int64_t i = global_index<kChunk>();
    if (i >= nf) return;
    if (pid[i] >= P.n_heavy) {
        pd[i] = T(0);
        return;
    }
    int c[3];
    cell_of(P, key[i], c);
    const Rec<T> me = pk[i];
    const T oi[3] = {me.x, me.y, me.z};
    T sW = T(0), sP = T(0), sR[3] = {0, 0, 0};
    visit4<T, D>(P, LF, i, fstart, PackSrc<T>{pk}, c, oi, [&](int j, const T d[3], T r2, uint32_t, const Rec<T>& q) {
        const T r0j = ld4(vk, j).w;
        if (r0j == P.rho0) return;  // a heavy neighbour
        const T W = wendland_W(P, pair_r(r2));
        const T rinv = T(1) / (r0j + q.w);
        sW += W * rinv;
        sP += P.c2 * q.w * W * rinv;
#pragma unroll
        for (int k = 0; k < D; ++k) sR[k] += W * d[k];
    });
    T gR = T(0);
#pragma unroll
    for (int k = 0; k < D; ++k) gR += P.gw[k] * sR[k];
    pd[i] = sW > T(0) ? (sP + gR) / sW : T(0);
}

// ---------------------------------------------------------------------------
// Momentum, Eq. (10) with p* of Eq. (8) (fluid) and Eq. (11) (walls),
// viscous term, penalty force Eqs. (13)-(15), gravity, second kick Eq. (22).
// Per fluid pair, with U_L - U_R = -(v_ij . r_ij)/r and F = W'(r)/r:
//   p* = [rho_i p_j + rho_j p_i + rho_i rho_j beta (U_L - U_R)]/(rho_i + rho_j)
//   dv_i/dt += m F/(rho_i rho_j) [-2 p* r_ij + 2 mu r^2/(r^2 + eta^2) v_ij].
// ---------------------------------------------------------------------------

// Waves per SIMD the FP32 momentum sweep is held to (80 VGPRs): one more
// wave in flight than its register count would give hides more of the
// neighbour loop's LDS latency than the few spilled registers cost.
template <typename T>
constexpr int kMomentumWaves = sizeof(T) == 4 ? 6 : 1;

template <typename T, int D, bool MP>
__global__ void __launch_bounds__(kBlock, kMomentumWaves<T>)
    k_momentum(Par<T> P, NbrMask LF, NbrMask LW, int64_t nf, int64_t nw, const int32_t* __restrict__ key,
               const int32_t* __restrict__ pid, const int32_t* __restrict__ fstart, const Rec<T>* __restrict__ pk,
               const Rec<T>* __restrict__ vk, const int32_t* __restrict__ wstart,
               const Rec<T>* __restrict__ wk, const Rec<T>* __restrict__ nk, T* __restrict__ acc,
               T* __restrict__ vel_out, Rec<T>* __restrict__ vk_out, T* __restrict__ sigma_next,
               const T* __restrict__ pd, int kick) {
    __shared__ Rec<T> stage[2 * kWaves * kStage];
    __shared__ int perm[kBlock];
    __shared__ int hist[16];
    const int64_t blk0 = (int64_t)logical_block() * kBlock;
    if (blk0 >= nf) return;  // the whole block is past the end
    const WaveSpan SB = span_of(P, key, blk0, (blk0 + kBlock < nf ? blk0 + kBlock : nf) - 1);
    const bool block_mode = LF.mask && SB.one_row;
    const int64_t i0 = block_mode ? regroup_block<T, D>(P, pk, blk0, nf, hist, perm) : blk0 + threadIdx.x;
    const int64_t ib = i0 - (threadIdx.x & 63);
    if (!block_mode && ib >= nf) return;  // the whole wave is past the end
    const bool act = i0 < nf;
    const int64_t i = act ? i0 : nf - 1;
    int c[3];
    cell_of(P, key[i], c);
    const Rec<T> me = pk[i];
    const Rec<T> mv = vk[i];
    const T oi[3] = {me.x, me.y, me.z};
    const T vi[3] = {mv.x, mv.y, mv.z};
    const T dri = me.w;
    const bool light = MP && pid[i] >= P.n_heavy;
    const T r0i = light ? P.rho0L : P.rho0;  // own reference density
    const T rho_i = r0i + dri;
    const T p_i = P.c2 * dri;
    const T inv_rho_i = T(1) / rho_i;
    const T m_rho_i = P.m * inv_rho_i;  // m_j / rho_i of a single-phase pair
    T A[3] = {0, 0, 0};
    // sigma of these positions, the next density update's sum (Eq. (4)):
    // every visited pair, self included, fluid then walls, as k_density sums it
    T s = T(0), comp = T(0);
    auto fluid = [&](int j, const T d[3], T r2, uint32_t, const Rec<T>& q, const Rec<T>& vj) {
        // no branch for r = 0 (the particle itself, or a coincident one): with
        // the reciprocal root taken of 1 there, every part of its force carries
        // r or d and adds an exact zero, and the velocity record is read
        // without waiting on r2
        T rinv;
        const T r = pair_r(r2, rinv);
        const KernelWF<T> k = wendland_WF(P, r);
        kahan_add(s, comp, k.W);
        const T F = k.F;
        const T drj = q.w;
        T r0j = MP ? vj.w : P.rho0;
        T p_j = P.c2 * drj;
        // two phases with cross_phase: a light particle sees a heavy neighbour
        // as a moving wall dummy (p* of Eq. (11), the light phase's EOS
        // density and mass), carrying the heavy particle's own pressure (1)
        // or the one extrapolated from its light neighbours (2); otherwise
        // each side keeps its own state
        const bool dummy = MP && P.cross_phase && light && r0j != r0i;
        T rho_j = r0j + drj;
        if (dummy) {
            if (P.cross_phase == 2) p_j = ldg(pd, j);
            r0j = r0i;
            rho_j = r0i + p_j * P.inv_c2;
        }
        const T vjk[3] = {vj.x, vj.y, vj.z};
        T dv[3];
        T vd = T(0);
#pragma unroll
        for (int k = 0; k < D; ++k) {
            dv[k] = vi[k] - vjk[k];
            vd += dv[k] * d[k];
        }
        const T jump = -vd * rinv;  // U_L - U_R
        const T beta = dummy ? T(0) : minv(T(3) * maxv(jump, T(0)), P.c);
        const T sum = rho_i + rho_j;
        const T qq = rcp(rho_j * sum);  // 1/(rho_j (rho_i + rho_j))
        const T pstar = (rho_i * p_j + rho_j * p_i + rho_i * rho_j * beta * jump) * (rho_j * qq);
        const T mr = MP ? r0j * P.vol * inv_rho_i : m_rho_i;
        const T coef = mr * F * (sum * qq);  // m_j F/(rho_i rho_j)
        const T visc = P.mu2 * r2 * rcp(r2 + P.eta2);
        const T cv = coef * visc, cp = T(-2) * coef * pstar;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            A[k] += cv * dv[k];
            A[k] += cp * d[k];
        }
    };
    auto fluid_g = [&](int j, const T d[3], T r2, uint32_t code, const Rec<T>& q) {
        fluid(j, d, r2, code, q, ld4(vk, j));
    };
    fluid_sweep<kStage, T, D>(P, LF, fstart, pk, vk, key, stage, block_mode, SB, act, ib, nf, i, c, oi, fluid,
                              fluid_g);
    if (!act) return;
    if (nw > 0 && (!LW.mask || LW.count[i] != 0))  // no wall neighbour: nothing to add
        visit_walls<T, D>(P, LW, i, wstart, wk, (P.penalty || light) ? nk : nullptr, c, oi,
                     [&](int, const T d[3], T r2, const Rec<T>& q, const Rec<T>& nw4) {
                         const T r = pair_r(r2);
                         const KernelWF<T> k = wendland_WF(P, r);
                         kahan_add(s, comp, k.W);
                         if (!(r2 > T(0))) return;
                         const T F = k.F;
                         const T p_w = q.w;
                         const T rho_w = r0i + p_w * P.inv_c2;  // the wall takes i's phase
                         const T sum = rho_i + rho_w;
                         const T qq = rcp(rho_w * sum);
                         const T pstar = (rho_i * p_w + rho_w * p_i) * (rho_w * qq);
                         const T mw = MP ? r0i * P.vol : P.m;
                         const T coef = mw * F * (sum * qq) * inv_rho_i;
                         const T visc = P.mu2 * r2 * rcp(r2 + P.eta2);
                         T pen = T(0);
                         T nv[3] = {0, 0, 0};
                         if (P.penalty || light) {
                             nv[0] = nw4.x;
                             nv[1] = nw4.y;
                             nv[2] = D == 3 ? nw4.z : T(0);
                             T proj = T(0);
#pragma unroll
                             for (int k = 0; k < D; ++k) proj += d[k] * nv[k];
                             const T ap = absv(proj);
                             const T delta = P.two_over_dx * ap;
                             if (delta < T(1)) {
                                 const T om = T(1) - delta;
                                 pen = -T(2) * P.gamma_p * om * om * absv(p_i) * ap;
                             }
                         }
#pragma unroll
                         for (int k = 0; k < D; ++k)
                             A[k] += coef * (visc * vi[k] - T(2) * pstar * d[k] + pen * nv[k]);
                     });
    T vn[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const T a = A[k] + P.g[k];
        acc[k * nf + i] = a;
        vn[k] = vi[k] + P.half_dt * a + P.fk[k];
        if (kick) vel_out[k * nf + i] = vn[k];
    }
    if (kick) vk_out[i] = Rec<T>{vn[0], vn[1], vn[2], r0i};
    sigma_next[i] = s;
}

// ---------------------------------------------------------------------------
// Neighbour masks, built once per step right after the sort: the culling of
// the stencil candidates happens here only, and every row's result is one
// coalesced store of two 64-bit words; the sweeps then visit the recorded
// pairs.  Queries with a row of more than 128 candidates get count -1 and
// walk the cells in the sweeps (counted in the status words).
// ---------------------------------------------------------------------------

template <typename T, int D>
__global__ void __launch_bounds__(kBlock)
    k_masks_fluid(Par<T> P, int64_t nf, int64_t nw, const int32_t* __restrict__ key,
                  const Rec<T>* __restrict__ pk, const int32_t* __restrict__ fstart,
                  const Rec<T>* __restrict__ wk, const int32_t* __restrict__ wstart,
                  const uint8_t* __restrict__ wnear, uint64_t* __restrict__ mf, int32_t* __restrict__ cf,
                  uint64_t* __restrict__ mw, int32_t* __restrict__ cw, uint32_t* __restrict__ status) {
    __shared__ Rec<T> stage_p[kBlock / 64][kStageM];
    const int64_t i0 = global_index<kChunk>();
    const int64_t ib = i0 - (threadIdx.x & 63);
    if (ib >= nf) return;  // the whole wave is past the end
    const bool act = i0 < nf;
    const int64_t i = act ? i0 : nf - 1;
    const int k = key[i];
    // cells without a wall particle among their neighbour cells (wnear,
    // built once at init) have no wall candidates: every wall row would be
    // skipped and no word written
    const bool near = nw > 0 && wnear[k] != 0;
    int c[3];
    cell_of(P, k, c);
    const Rec<T> me = pk[i];
    const T oi[3] = {me.x, me.y, me.z};
    const WaveSpan S = wave_span(P, key, ib, nf);
    int n = 0;
    if (S.one_row)
        n = build_mask_staged<T, D, kStageM>(P, fstart, pk, (SPH_LDS Rec<T>*)stage_p[threadIdx.x >> 6], S, act,
                                            c, oi, mf, nf, i);
    else if (act)
        n = build_mask<T, D>(P, fstart, PackSrc<T>{pk}, c, oi, mf, nf, i);
    if (!act) return;
    cf[i] = n;
    int m = 0;
    if (near) m = build_mask<T, D>(P, wstart, PackSrc<T>{wk}, c, oi, mw, nf, i);
    cw[i] = m;
    if (n < 0 || m < 0) atomicAdd(&status[SPH_STATUS_LIST_OVERFLOW], 1u);
}

template <typename T, int D>
__global__ void __launch_bounds__(kBlock)
    k_masks_wall(Par<T> P, int64_t nf, int64_t nw, const int32_t* __restrict__ wkey,
                 const Rec<T>* __restrict__ wk, const Rec<T>* __restrict__ pk,
                 const int32_t* __restrict__ fstart, uint64_t* __restrict__ m,
                 int32_t* __restrict__ cnt, uint32_t* __restrict__ status) {
    const int64_t w = global_index<kChunk>();
    if (w >= nw) return;
    int c[3];
    cell_of(P, wkey[w], c);
    const Rec<T> me = wk[w];
    const T ow[3] = {me.x, me.y, me.z};
    int n = 0;
    if (nf > 0) n = build_mask<T, D>(P, fstart, PackSrc<T>{pk}, c, ow, m, nw, w);
    cnt[w] = n;
    if (n < 0) atomicAdd(&status[SPH_STATUS_LIST_OVERFLOW], 1u);
}

// ---------------------------------------------------------------------------
// FP64 diagnostics: per-block partials, then one block in fixed order.
// ---------------------------------------------------------------------------

// Exact FP64 particle mass and body force of the reductions (by value).
struct DiagC {
    double m, m_light;  // heavy (or only) and light phase particle masses
    double g[3];
};


template <typename T, int D>
__global__ void __launch_bounds__(kBlock)
    k_diag_partial(Par<T> P, GridD G, DiagC K, int64_t nf,
                   const int32_t* __restrict__ key, const int32_t* __restrict__ pid, const T* __restrict__ off,
                   const T* __restrict__ vel, const T* __restrict__ drho, double* __restrict__ part) {
    __shared__ double red[kDiagVals][kBlock];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double v[kDiagVals] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (i < nf) {
        int c[3];
        cell_of(P, key[i], c);
        double v2 = 0.0, gx = 0.0;
        const double m = (P.two_phase && pid[i] >= P.n_heavy) ? K.m_light : K.m;
        bool finite = isfinite((double)drho[i]);
        for (int k = 0; k < D; ++k) {
            const double vk = (double)vel[k * nf + i] + G.V[k];
            const double xk = G.lo[k] + (double)c[k] * G.L + (double)off[k * nf + i] + G.X[k];
            finite = finite && isfinite(vk) && isfinite(xk);
            v[1 + k] = m * vk;
            v2 += vk * vk;
            gx += K.g[k] * xk;
        }
        v[0] = m;
        v[4] = 0.5 * m * v2;
        v[5] = -m * gx;
        v[6] = sqrt(v2);
        v[7] = finite ? 0.0 : 1.0;
    }
    for (int k = 0; k < kDiagVals; ++k) red[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int k = 0; k < kDiagVals; ++k) {
                if (k == 6)
                    red[k][threadIdx.x] = fmax(red[k][threadIdx.x], red[k][threadIdx.x + o]);
                else
                    red[k][threadIdx.x] += red[k][threadIdx.x + o];
            }
        __syncthreads();
    }
    if (threadIdx.x < kDiagVals) part[(int64_t)blockIdx.x * kDiagVals + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void __launch_bounds__(kBlock)
    k_diag_final(const double* __restrict__ part, int nblocks, double* __restrict__ diag,
                 uint32_t* __restrict__ status) {
    __shared__ double red[kDiagVals][kBlock];
    double v[kDiagVals] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblocks; b += kBlock)
        for (int k = 0; k < kDiagVals; ++k) {
            const double x = part[(int64_t)b * kDiagVals + k];
            v[k] = k == 6 ? fmax(v[k], x) : v[k] + x;
        }
    for (int k = 0; k < kDiagVals; ++k) red[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int k = 0; k < kDiagVals; ++k) {
                if (k == 6)
                    red[k][threadIdx.x] = fmax(red[k][threadIdx.x], red[k][threadIdx.x + o]);
                else
                    red[k][threadIdx.x] += red[k][threadIdx.x + o];
            }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        diag[SPH_DIAG_MASS] = red[0][0];
        diag[SPH_DIAG_MOM + 0] = red[1][0];
        diag[SPH_DIAG_MOM + 1] = red[2][0];
        diag[SPH_DIAG_MOM + 2] = red[3][0];
        diag[SPH_DIAG_EKIN] = red[4][0];
        diag[SPH_DIAG_EPOT] = red[5][0];
        diag[SPH_DIAG_VMAX] = red[6][0];
        if (red[7][0] > 0.0) atomicAdd(&status[SPH_STATUS_NONFINITE], (uint32_t)red[7][0]);
    }
}

__global__ void k_count_step(double* diag) {
    if (threadIdx.x == 0 && blockIdx.x == 0) diag[SPH_DIAG_STEPS] += 1.0;
}

// ---------------------------------------------------------------------------
// Export in particle-id order (doubles).
// ---------------------------------------------------------------------------

template <typename T, int D>
__global__ void __launch_bounds__(kBlock)
    k_export(Par<T> P, GridD G, int64_t nf, const int32_t* __restrict__ key,
             const int32_t* __restrict__ pid, const T* __restrict__ off, const T* __restrict__ vel,
             const T* __restrict__ drho, const T* __restrict__ acc, double* __restrict__ pos_o,
             double* __restrict__ vel_o, double* __restrict__ rho_o, double* __restrict__ acc_o) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nf) return;
    const int64_t p = pid[i];
    int c[3];
    cell_of(P, key[i], c);
    for (int k = 0; k < D; ++k) {
        if (pos_o) pos_o[k * nf + p] = G.lo[k] + (double)c[k] * G.L + (double)off[k * nf + i] + G.X[k];
        if (vel_o) vel_o[k * nf + p] = (double)vel[k * nf + i] + G.V[k];
        if (acc_o) acc_o[k * nf + p] = (double)acc[k * nf + i];
    }
    if (rho_o) rho_o[p] = (double)ref_density(P, (int)p) + (double)drho[i];
}

template <typename T, int D>
__global__ void __launch_bounds__(kBlock)
    k_export_walls(Par<T> P, GridD G, int64_t nw, const int32_t* __restrict__ wkey,
                   const int32_t* __restrict__ wpid, const T* __restrict__ woff,
                   const T* __restrict__ pw, const T* __restrict__ nrm, double* __restrict__ pw_o,
                   double* __restrict__ nrm_o, double* __restrict__ pos_o) {
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= nw) return;
    const int64_t p = wpid[w];
    int c[3];
    cell_of(P, wkey[w], c);
    if (pw_o) pw_o[p] = (double)pw[w];
    for (int k = 0; k < D; ++k) {
        if (nrm_o) nrm_o[k * nw + p] = (double)nrm[k * nw + w];
        if (pos_o) pos_o[k * nw + p] = G.lo[k] + (double)c[k] * G.L + (double)woff[k * nw + w] + G.X[k];
    }
}

// Neighbour sets as the sweeps see them (test and inspection aid).
template <typename T, int D>
__global__ void __launch_bounds__(kBlock)
    k_neighbours(Par<T> P, int which, int64_t nf, int64_t nw, const int32_t* __restrict__ key,
                 const int32_t* __restrict__ pid, const T* __restrict__ off,
                 const int32_t* __restrict__ fstart, const int32_t* __restrict__ wkey,
                 const int32_t* __restrict__ wpid, const T* __restrict__ woff,
                 const int32_t* __restrict__ wstart, const int64_t* __restrict__ offset,
                 int32_t* __restrict__ count, int32_t* __restrict__ list, int64_t list_len) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nq = which == 0 ? nf : nw;
    if (i >= nq) return;
    const int32_t* qkey = which == 0 ? key : wkey;
    const T* qoff = which == 0 ? off : woff;
    const int32_t qid = which == 0 ? pid[i] : wpid[i];
    int c[3];
    cell_of(P, qkey[i], c);
    const T oi[3] = {qoff[i], qoff[nq + i], D == 3 ? qoff[2 * nq + i] : T(0)};
    int cnt = 0;
    int64_t base = list ? offset[qid] : 0;
    if (nf > 0)
        for_neighbours<T, D>(P, fstart, off, off + nf, off + 2 * nf, c, oi, [&](int j, const T*, T, uint32_t) {
            if (list && base + cnt >= 0 && base + cnt < list_len) list[base + cnt] = pid[j];
            ++cnt;
        });
    if (which == 0 && nw > 0)
        for_neighbours<T, D>(P, wstart, woff, woff + nw, woff + 2 * nw, c, oi,
                             [&](int j, const T*, T, uint32_t) {
                                 if (list && base + cnt >= 0 && base + cnt < list_len)
                                     list[base + cnt] = (int32_t)nf + wpid[j];
                                 ++cnt;
                             });
    count[qid] = cnt;
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

// Sort n keys into cell order: start table + permutation (scratch.perm).
// The histogram's slot of each key goes to scratch.perm, the placement by
// slot to scratch.slot, and the in-cell ranking back to scratch.perm, by x
// offset when ox (the set's x offsets, precision of d) is given.
int sort_keys(const sph_desc* d, const Scratch& s, const int32_t* key, int64_t n, int32_t* start,
              hipStream_t st, const void* ox = nullptr) {
    const int64_t nc = d->n_cells;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(nc)), dim3(kBlock), 0, st, s.count, nc, 0);
    SPH_LAUNCH_CHECK();
    if (n > 0) {
        hipLaunchKernelGGL(k_hist, dim3(grid_for(n)), dim3(kBlock), 0, st, key, n, s.count, s.perm);
        SPH_LAUNCH_CHECK();
    }
    const int ntiles = (int)((nc + kScanTile - 1) / kScanTile);
    hipLaunchKernelGGL(k_scan_reduce, dim3(ntiles), dim3(kScanThreads), 0, st, s.count, nc, s.tiles);
    SPH_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kScanThreads), 0, st, s.tiles, ntiles);
    SPH_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scan_down, dim3(ntiles), dim3(kScanThreads), 0, st, s.count, nc, s.tiles,
                       start, (int32_t)n);
    SPH_LAUNCH_CHECK();
    if (n > 0) {
        hipLaunchKernelGGL(k_place, dim3(grid_for(n)), dim3(kBlock), 0, st, key, s.perm, n, start,
                           s.slot);
        SPH_LAUNCH_CHECK();
        if (d->precision == SPH_F64)
            hipLaunchKernelGGL(k_cellrank<double>, dim3(grid_for(n)), dim3(kBlock), 0, st, key, start, s.slot, n,
                               (const double*)ox, s.perm);
        else
            hipLaunchKernelGGL(k_cellrank<float>, dim3(grid_for(n)), dim3(kBlock), 0, st, key, start, s.slot, n,
                               (const float*)ox, s.perm);
        SPH_LAUNCH_CHECK();
    }
    return SPH_OK;
}

template <typename T, int D>
int build_cells_t(const sph_desc* d, sph_buffers* b, hipStream_t st) {
    const Scratch s = layout(d, b->n_fluid, b->n_wall, b->scratch);
    const int64_t n = b->n_fluid;
    int rc = sort_keys(d, s, b->key[1], n, b->fstart, st, b->off[1]);
    if (rc) return rc;
    if (n > 0) {
        const int sv = b->sel_vel, sr = b->sel_rho;
        hipLaunchKernelGGL((k_gather_fluid<T, D>), dim3(grid_for(n)), dim3(kBlock), 0, st, make_par<T>(d), s.perm, n,
                           b->key[1], b->pid[1], (const T*)b->off[1], (const T*)b->vel[sv],
                           (const T*)b->rho[sr], b->key[0], b->pid[0], (T*)b->off[0],
                           (T*)b->vel[1 - sv], (T*)b->rho[1 - sr], (Rec<T>*)s.pk[1 - sr],
                           (Rec<T>*)s.vk[1 - sv]);
        SPH_LAUNCH_CHECK();
    }
    b->sel_vel = 1 - b->sel_vel;
    b->sel_rho = 1 - b->sel_rho;
    b->sigma_ready = 0;
    if (b->nbr_ff) {
        const Par<T> P = make_par<T>(d);
        const Rec<T>* pk = (const Rec<T>*)s.pk[b->sel_rho];
        if (n > 0) {
            hipLaunchKernelGGL((k_masks_fluid<T, D>), dim3(grid_for(n)), dim3(kBlock), 0, st, P, n, b->n_wall,
                               b->key[0], pk, b->fstart, (const Rec<T>*)s.wk, b->wstart, s.wnear,
                               b->nbr_ff, b->cnt_ff, b->nbr_fw, b->cnt_fw, b->status);
            SPH_LAUNCH_CHECK();
        }
        if (b->n_wall > 0) {
            hipLaunchKernelGGL((k_masks_wall<T, D>), dim3(grid_for(b->n_wall)), dim3(kBlock), 0, st, P, n,
                               b->n_wall, b->wkey, (const Rec<T>*)s.wk, pk, b->fstart,
                               b->nbr_wf, b->cnt_wf, b->status);
            SPH_LAUNCH_CHECK();
        }
    }
    return SPH_OK;
}

template <typename T, int D>
int density_t(const sph_desc* d, sph_buffers* b, hipStream_t st) {
    const int64_t nf = b->n_fluid, nw = b->n_wall;
    const bool ready = b->sigma_ready != 0;
    b->sigma_ready = 0;  // the drift moves the positions it was summed at
    const int64_t n = b->nstep++;
    if (nf == 0) return SPH_OK;
    Par<T> P = make_par<T>(d);
    if (moving(d)) {  // half kick in the tank frame: + X'(t_n) - Vh
        double Vh[3];
        drift_velocity(d, n, Vh);
        const Motion m = motion_at(d, n);
        for (int k = 0; k < 3; ++k) P.fk[k] = T(m.V[k] - Vh[k]);
    }
    const Scratch s = layout(d, nf, nw, b->scratch);
    hipLaunchKernelGGL((k_density<T, D>), dim3(grid_for(nf)), dim3(kBlock), 0, st, P, mask_ff(b),
                       mask_fw(b), nf, nw,
                       b->key[0], b->pid[0], (const T*)b->off[0], b->fstart, (const T*)b->woff,
                       b->wstart, (T*)b->vel[b->sel_vel], (T*)b->rho[b->sel_rho],
                       (const T*)b->acc, b->key[1], b->pid[1], (T*)b->off[1], (T*)b->sigma_out,
                       ready ? (const T*)s.sig : nullptr, (Rec<T>*)s.pk[b->sel_rho],
                       (Rec<T>*)s.vk[b->sel_vel], b->status);
    SPH_LAUNCH_CHECK();
    return SPH_OK;
}

template <typename T, int D>
int wall_bc_t(const sph_desc* d, sph_buffers* b, hipStream_t st, bool probe = true) {
    const int64_t nf = b->n_fluid, nw = b->n_wall;
    if (nw == 0) return SPH_OK;
    Par<T> P = make_par<T>(d);
    if (moving(d)) {  // Eq. (12) with a_w = a_wall + X''(t)
        const Motion m = motion_at(d, b->nstep);
        for (int k = 0; k < 3; ++k) P.gw[k] = T(d->g[k] - d->a_wall[k] - m.A[k]);
    }
    const Scratch s = layout(d, nf, nw, b->scratch);
    if (d->two_phase)
        hipLaunchKernelGGL((k_wall_bc<T, D, true>), dim3(grid_for(nw)), dim3(kBlock), 0, st, P, mask_wf(b), nf,
                           nw, b->wkey, b->fstart, (const Rec<T>*)s.pk[b->sel_rho],
                           (const Rec<T>*)s.vk[b->sel_vel], (Rec<T>*)s.wk, (T*)b->pw);
    else
        hipLaunchKernelGGL((k_wall_bc<T, D, false>), dim3(grid_for(nw)), dim3(kBlock), 0, st, P, mask_wf(b), nf,
                           nw, b->wkey, b->fstart, (const Rec<T>*)s.pk[b->sel_rho],
                           (const Rec<T>*)s.vk[b->sel_vel], (Rec<T>*)s.wk, (T*)b->pw);
    SPH_LAUNCH_CHECK();
    if (probe && b->n_probe > 0) {
        hipLaunchKernelGGL((k_probe<T>), dim3(1), dim3(kBlock), 0, st, (const T*)b->pw, s.winv, nw,
                           b->probe, b->n_probe, d->dt, b->diag);
        SPH_LAUNCH_CHECK();
    }
    return SPH_OK;
}

template <typename T, int D>
int forces_t(const sph_desc* d, sph_buffers* b, unsigned which, hipStream_t st) {
    const int64_t nf = b->n_fluid, nw = b->n_wall;
    Par<T> P = make_par<T>(d);
    if (moving(d) && !(which & SPH_NO_KICK)) {  // second kick in the tank frame: + Vh - X'(t_{n+1})
        double Vh[3];
        drift_velocity(d, b->nstep - 1, Vh);
        const Motion m = motion_at(d, b->nstep);
        for (int k = 0; k < 3; ++k) P.fk[k] = T(Vh[k] - m.V[k]);
    }
    const int sv = b->sel_vel, sr = b->sel_rho;
    const Scratch s = layout(d, nf, nw, b->scratch);
    const Rec<T>* wk = (const Rec<T>*)s.wk;
    if (which & SPH_CONTINUITY) {
        if (nf > 0) {
            auto kern = d->two_phase ? k_continuity<T, D, true> : k_continuity<T, D, false>;
            hipLaunchKernelGGL(kern, dim3(grid_for(nf)), dim3(kBlock), 0, st, P,
                               mask_ff(b), mask_fw(b), nf, nw, b->key[0], b->pid[0], b->fstart,
                               (const Rec<T>*)s.pk[sr], (const Rec<T>*)s.vk[sv], b->wstart, wk,
                               (T*)b->rho[1 - sr], (Rec<T>*)s.pk[1 - sr]);
            SPH_LAUNCH_CHECK();
        }
        b->sel_rho = 1 - sr;
    } else {
        const int kick = (which & SPH_NO_KICK) ? 0 : 1;
        const bool dummies = d->two_phase && d->cross_phase == 2;
        if (nf > 0 && dummies) {  // the heavy particles' dummy pressures, g - a_w of the tank at nstep
            Par<T> Q = P;
            const Motion m = motion_at(d, b->nstep);
            for (int k = 0; k < 3; ++k) Q.gw[k] = T(d->g[k] - d->a_wall[k] - (moving(d) ? m.A[k] : 0.0));
            hipLaunchKernelGGL((k_dummy_pressure<T, D>), dim3(grid_for(nf)), dim3(kBlock), 0, st, Q, mask_ff(b),
                               nf, b->key[0], b->pid[0], b->fstart, (const Rec<T>*)s.pk[sr],
                               (const Rec<T>*)s.vk[sv], (T*)s.pd);
            SPH_LAUNCH_CHECK();
        }
        if (nf > 0) {
            auto kern = d->two_phase ? k_momentum<T, D, true> : k_momentum<T, D, false>;
            hipLaunchKernelGGL(kern, dim3(grid_for(nf)), dim3(kBlock), 0, st, P,
                               mask_ff(b), mask_fw(b), nf, nw, b->key[0], b->pid[0], b->fstart,
                               (const Rec<T>*)s.pk[sr], (const Rec<T>*)s.vk[sv], b->wstart, wk,
                               (const Rec<T>*)s.nk, (T*)b->acc, (T*)b->vel[1 - sv],
                               (Rec<T>*)s.vk[1 - sv], (T*)s.sig, dummies ? (const T*)s.pd : nullptr, kick);
            SPH_LAUNCH_CHECK();
        }
        if (kick) b->sel_vel = 1 - sv;
        b->sigma_ready = 1;
    }
    return SPH_OK;
}

template <typename T, int D>
int init_t(const sph_desc* d, sph_buffers* b, const double* fpos, const double* fvel,
           const double* frho, const double* wpos, hipStream_t st) {
    const int64_t nf = b->n_fluid, nw = b->n_wall;
    const Scratch s = layout(d, nf, nw, b->scratch);
    b->nstep = 0;
    const GridD G = make_grid_at(d, 0);  // inputs are fixed-frame positions at t = 0
    const Par<T> P = make_par<T>(d);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(kBlock), 0, st, (int32_t*)b->status,
                       (int64_t)SPH_STATUS_LEN, 0);
    SPH_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(kBlock), 0, st, b->diag, (int64_t)SPH_DIAG_LEN, 0.0);
    SPH_LAUNCH_CHECK();
    // walls: cells, one sort, normals
    if (nw > 0) {
        hipLaunchKernelGGL((k_to_cells<T, D>), dim3(grid_for(nw)), dim3(kBlock), 0, st, wpos, nw, G,
                           s.wkey0, (T*)s.woff0, b->status);
        SPH_LAUNCH_CHECK();
    }
    int rc = sort_keys(d, s, s.wkey0, nw, b->wstart, st);
    if (rc) return rc;
    if (nw > 0) {
        hipLaunchKernelGGL((k_gather_wall<T, D>), dim3(grid_for(nw)), dim3(kBlock), 0, st, s.perm, nw,
                           s.wkey0, (const T*)s.woff0, b->wkey, b->wpid, (T*)b->woff, s.winv);
        SPH_LAUNCH_CHECK();
        hipLaunchKernelGGL((k_normals<T, D>), dim3(grid_for(nw)), dim3(kBlock), 0, st, P, nw, b->wkey,
                           (const T*)b->woff, b->wstart, (T*)b->nrm);
        SPH_LAUNCH_CHECK();
        hipLaunchKernelGGL((k_pack_walls<T, D>), dim3(grid_for(nw)), dim3(kBlock), 0, st, nw,
                           (const T*)b->woff, (const T*)b->nrm, (Rec<T>*)s.wk, (Rec<T>*)s.nk);
        SPH_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL((k_wall_near<T, D>), dim3(grid_for(d->n_cells)), dim3(kBlock), 0, st, P, d->n_cells,
                       b->wstart, s.wnear);
    SPH_LAUNCH_CHECK();
    // fluid: cells of the initial positions into copy 1, state into the
    // current copies, then the sort brings everything to copy 0.
    b->sel_vel = 0;
    b->sel_rho = 0;
    b->sigma_ready = 0;
    if (nf > 0) {
        hipLaunchKernelGGL((k_to_cells<T, D>), dim3(grid_for(nf)), dim3(kBlock), 0, st, fpos, nf, G,
                           b->key[1], (T*)b->off[1], b->status);
        SPH_LAUNCH_CHECK();
        hipLaunchKernelGGL((k_init_state<T, D>), dim3(grid_for(nf)), dim3(kBlock), 0, st, P, G, nf,
                           fvel, frho, b->pid[1], (T*)b->vel[0], (T*)b->rho[0]);
        SPH_LAUNCH_CHECK();
    }
    rc = build_cells_t<T, D>(d, b, st);
    if (rc) return rc;
    rc = wall_bc_t<T, D>(d, b, st, false);  // p_w of the initial state, not integrated
    if (rc) return rc;
    return forces_t<T, D>(d, b, SPH_MOMENTUM | SPH_NO_KICK, st);
}

template <typename T, int D>
int step_t(const sph_desc* d, sph_buffers* b, int nsteps, hipStream_t st) {
    for (int n = 0; n < nsteps; ++n) {
        int rc = density_t<T, D>(d, b, st);
        if (!rc) rc = build_cells_t<T, D>(d, b, st);
        if (!rc) rc = wall_bc_t<T, D>(d, b, st);
        if (!rc) rc = forces_t<T, D>(d, b, SPH_CONTINUITY, st);
        if (!rc) rc = forces_t<T, D>(d, b, SPH_MOMENTUM, st);
        if (rc) return rc;
        hipLaunchKernelGGL(k_count_step, dim3(1), dim3(64), 0, st, b->diag);
        SPH_LAUNCH_CHECK();
    }
    return SPH_OK;
}

// Up to kMaxCopies device-to-device copies of 4-byte words in one launch
// (blockIdx.y picks the copy).
constexpr int kMaxCopies = 16;
struct CopyList {
    const uint32_t* src[kMaxCopies];
    uint32_t* dst[kMaxCopies];
    int64_t words[kMaxCopies];
};

__global__ void __launch_bounds__(kBlock) k_copy_words(CopyList L) {
    const int c = blockIdx.y;
    const int64_t n = L.words[c];
    const uint32_t* __restrict__ src = L.src[c];
    uint32_t* __restrict__ dst = L.dst[c];
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        dst[k] = src[k];
}

// Adds a copy of n bytes (a multiple of 4) to the list, skipped when either
// side is absent or n is 0.
inline void add_copy(CopyList& L, int& m, const void* dst, const void* src, size_t n) {
    if (!dst || !src || n == 0) return;
    L.src[m] = (const uint32_t*)src;
    L.dst[m] = (uint32_t*)dst;
    L.words[m] = (int64_t)(n / 4);
    ++m;
}

template <typename T, int D>
int step_frame_t(const sph_desc* d, sph_buffers* b, void* sigma_cur, sph_frame* nx, hipStream_t st) {
    const int64_t nf = b->n_fluid, nw = b->n_wall;
    const size_t ts = sizeof(T);
    void* keep = b->sigma_out;
    b->sigma_out = sigma_cur;
    int rc = density_t<T, D>(d, b, st);
    b->sigma_out = keep;
    if (!rc) rc = build_cells_t<T, D>(d, b, st);
    if (rc) return rc;
    // Every array the frame records stays as it is from here to the end of
    // the step (the sweeps write the other velocity and density copies), so
    // all of them are copied in one launch at the end.
    const void* vh = b->vel[b->sel_vel];
    const void* rt = b->rho[b->sel_rho];
    if (!rc) rc = wall_bc_t<T, D>(d, b, st);
    if (!rc) rc = forces_t<T, D>(d, b, SPH_CONTINUITY, st);
    const void* rho1 = b->rho[b->sel_rho];
    if (!rc) rc = forces_t<T, D>(d, b, SPH_MOMENTUM, st);
    if (rc) return rc;
    CopyList L;
    int m = 0;
    add_copy(L, m, nx->key, b->key[0], 4 * (size_t)nf);
    add_copy(L, m, nx->pid, b->pid[0], 4 * (size_t)nf);
    add_copy(L, m, nx->off, b->off[0], ts * D * (size_t)nf);
    add_copy(L, m, nx->fstart, b->fstart, 4 * (size_t)(d->n_cells + 1));
    add_copy(L, m, nx->vh, vh, ts * D * (size_t)nf);
    add_copy(L, m, nx->rt, rt, ts * (size_t)nf);
    add_copy(L, m, nx->pw, b->pw, ts * (size_t)nw);
    add_copy(L, m, nx->rho, rho1, ts * (size_t)nf);
    if (b->nbr_ff && nx->nbr_ff && nx->nbr_fw && nx->nbr_wf && nx->cnt_ff && nx->cnt_fw && nx->cnt_wf) {
        const size_t rows = d->dim == 3 ? 9 : 3;
        const size_t wf = 8 * 2 * rows * (size_t)nf, ww = 8 * 2 * rows * (size_t)nw;
        add_copy(L, m, nx->nbr_ff, b->nbr_ff, wf);
        add_copy(L, m, nx->nbr_fw, b->nbr_fw, wf);
        add_copy(L, m, nx->nbr_wf, b->nbr_wf, ww);
        add_copy(L, m, nx->cnt_ff, b->cnt_ff, 4 * (size_t)nf);
        add_copy(L, m, nx->cnt_fw, b->cnt_fw, 4 * (size_t)nf);
        add_copy(L, m, nx->cnt_wf, b->cnt_wf, 4 * (size_t)nw);
    }
    if (m > 0) {
        int64_t most = 0;
        for (int k = 0; k < m; ++k) most = L.words[k] > most ? L.words[k] : most;
        const int gx = (int)((most + kBlock - 1) / kBlock < 2048 ? (most + kBlock - 1) / kBlock : 2048);
        hipLaunchKernelGGL(k_copy_words, dim3(gx > 0 ? gx : 1, m), dim3(kBlock), 0, st, L);
        SPH_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_count_step, dim3(1), dim3(64), 0, st, b->diag);
    SPH_LAUNCH_CHECK();
    nx->nstep = b->nstep;
    return SPH_OK;
}

// The reductions of sph_diag with the per-block partials (kDiagVals doubles
// per block of kBlock particles) in `part`.
template <typename T, int D>
int diag_impl(const sph_desc* d, sph_buffers* b, double* part, hipStream_t st) {
    const int64_t nf = b->n_fluid;
    const int nb = nf > 0 ? grid_for(nf) : 0;
    if (nb > 0) {
        DiagC K;
        const double vol = d->dim == 2 ? d->dx * d->dx : d->dx * d->dx * d->dx;
        K.m = d->rho0 * vol;
        K.m_light = (d->two_phase ? d->rho0_light : d->rho0) * vol;
        for (int k = 0; k < 3; ++k) K.g[k] = d->g[k];
        hipLaunchKernelGGL((k_diag_partial<T, D>), dim3(nb), dim3(kBlock), 0, st, make_par<T>(d),
                           make_grid_at(d, b->nstep), K, nf, b->key[0], b->pid[0], (const T*)b->off[0],
                           (const T*)b->vel[b->sel_vel], (const T*)b->rho[b->sel_rho], part);
        SPH_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(kBlock), 0, st, part, nb, b->diag, b->status);
    SPH_LAUNCH_CHECK();
    return SPH_OK;
}

template <typename T, int D>
int diag_t(const sph_desc* d, sph_buffers* b, hipStream_t st) {
    return diag_impl<T, D>(d, b, layout(d, b->n_fluid, b->n_wall, b->scratch).part, st);
}

template <typename T, int D>
int diag_static_t(const sph_desc* d, sph_buffers* b, double* part, hipStream_t st) {
    return diag_impl<T, D>(d, b, part, st);
}

template <typename T, int D>
int export_t(const sph_desc* d, const sph_buffers* b, double* pos, double* vel, double* rho,
             double* acc, hipStream_t st) {
    const int64_t nf = b->n_fluid;
    if (nf == 0) return SPH_OK;
    hipLaunchKernelGGL((k_export<T, D>), dim3(grid_for(nf)), dim3(kBlock), 0, st, make_par<T>(d),
                       make_grid_at(d, b->nstep), nf, b->key[0], b->pid[0], (const T*)b->off[0],
                       (const T*)b->vel[b->sel_vel], (const T*)b->rho[b->sel_rho],
                       (const T*)b->acc, pos, vel, rho, acc);
    SPH_LAUNCH_CHECK();
    return SPH_OK;
}

template <typename T, int D>
int export_walls_t(const sph_desc* d, const sph_buffers* b, double* pw, double* nrm, double* pos,
                   hipStream_t st) {
    const int64_t nw = b->n_wall;
    if (nw == 0) return SPH_OK;
    hipLaunchKernelGGL((k_export_walls<T, D>), dim3(grid_for(nw)), dim3(kBlock), 0, st,
                       make_par<T>(d), make_grid_at(d, b->nstep), nw, b->wkey, b->wpid,
                       (const T*)b->woff, (const T*)b->pw, (const T*)b->nrm, pw, nrm, pos);
    SPH_LAUNCH_CHECK();
    return SPH_OK;
}

template <typename T, int D>
int neighbours_t(const sph_desc* d, const sph_buffers* b, int which, const int64_t* offset,
                 int32_t* count, int32_t* list, int64_t list_len, hipStream_t st) {
    const int64_t nq = which == 0 ? b->n_fluid : b->n_wall;
    if (nq == 0) return SPH_OK;
    hipLaunchKernelGGL((k_neighbours<T, D>), dim3(grid_for(nq)), dim3(kBlock), 0, st, make_par<T>(d),
                       which, b->n_fluid, b->n_wall, b->key[0], b->pid[0], (const T*)b->off[0],
                       b->fstart, b->wkey, b->wpid, (const T*)b->woff, b->wstart, offset, count,
                       list, list_len);
    SPH_LAUNCH_CHECK();
    return SPH_OK;
}

// Dispatch on precision and dimension.
#define SPH_DISPATCH(fn, ...)                                                          \
    (d->precision == SPH_F32 ? (d->dim == 2 ? fn<float, 2>(__VA_ARGS__) : fn<float, 3>(__VA_ARGS__)) \
                             : (d->dim == 2 ? fn<double, 2>(__VA_ARGS__) : fn<double, 3>(__VA_ARGS__)))

}  // namespace

// Workspace of sph_diag_noalloc: the per-block partials of the reductions,
// in a device array that the library holds for the life of the process
// (one copy per GPU), so that call allocates nothing.  Host code never
// passes this name to a kernel (on the host it is only a stand-in for the
// symbol): it passes the address hipGetSymbolAddress returns for the
// current device, looked up once per device.
static __device__ __align__(256) unsigned char scratch[SPH_DIAG_NOALLOC_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the
// first call made with that device current).
int static_scratch(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SPH_ERR_LAUNCH;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SPH_ERR_LAUNCH;
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return SPH_OK;
}

}  // namespace

extern "C" {

int sph_configure(sph_desc* d) {
    if (!d) return SPH_ERR_ARG;
    if (d->dim != 2 && d->dim != 3) return SPH_ERR_CONFIG;
    if (d->precision != SPH_F32 && d->precision != SPH_F64) return SPH_ERR_CONFIG;
    if (!(d->h > 0.0) || !(d->dx > 0.0) || !(d->c0 > 0.0) || !(d->rho0 > 0.0) || !(d->dt > 0.0))
        return SPH_ERR_CONFIG;
    if (d->two_phase != 0 && d->two_phase != 1) return SPH_ERR_CONFIG;
    if (d->cross_phase < 0 || d->cross_phase > 2) return SPH_ERR_CONFIG;
    if (d->two_phase && (!(d->rho0_light > 0.0) || d->n_heavy < 0 || d->n_heavy > (int64_t)INT32_MAX))
        return SPH_ERR_CONFIG;
    if (!std::isfinite(d->motion_freq) || d->motion_freq < 0.0) return SPH_ERR_CONFIG;
    double amp = 0.0;
    for (int k = 0; k < 3; ++k) {
        if (!std::isfinite(d->motion_amp[k])) return SPH_ERR_CONFIG;
        amp += d->motion_amp[k] * d->motion_amp[k];
    }
    // time step bound, Eqs. (23)-(24) with U_max = c0/10; the body force
    // bound takes |g| plus the largest tank acceleration
    double gn = 0.0;
    for (int k = 0; k < 3; ++k) gn += d->g[k] * d->g[k];
    const double w = 2.0 * M_PI * d->motion_freq;
    gn = std::sqrt(gn) + std::sqrt(amp) * w * w;
    double dtmax = 0.25 * d->h / (1.1 * d->c0);
    if (gn > 0.0) dtmax = std::fmin(dtmax, 0.25 * std::sqrt(d->h / gn));
    if (d->dt > dtmax * 1.01) return SPH_ERR_CONFIG;  // 1 % slack: dt held fixed while c0 is varied
    // cell edge: 2h rounded to T, raised until L^2 >= rc2 so that every pair
    // lies in adjacent cells
    double L;
    if (d->precision == SPH_F32) {
        float Lf = (float)(2.0 * d->h);
        const float rc2 = (float)(4.0 * d->h * d->h);
        while (Lf * Lf < rc2 || (double)Lf < 2.0 * d->h) Lf = std::nextafter(Lf, 1e30f);
        L = Lf;
    } else {
        L = 2.0 * d->h;
    }
    d->cell = L;
    int64_t nc = 1;
    for (int k = 0; k < 3; ++k) {
        if (k < d->dim) {
            if (!(d->hi[k] > d->lo[k])) return SPH_ERR_CONFIG;
            const double n = std::ceil((d->hi[k] - d->lo[k]) / L);
            if (n > 1e9) return SPH_ERR_CONFIG;
            d->grid[k] = (int32_t)(n < 1 ? 1 : n);
        } else {
            d->grid[k] = 1;
        }
        nc *= d->grid[k];
        if (nc > (int64_t)INT32_MAX - 2) return SPH_ERR_CONFIG;
    }
    d->n_cells = nc;
    // sigma0: sum_j W over a full lattice of spacing dx around one site
    const double h = d->h;
    const double alpha = d->dim == 2 ? 7.0 / (4.0 * M_PI * h * h) : 21.0 / (16.0 * M_PI * h * h * h);
    const int R = (int)std::ceil(2.0 * h / d->dx) + 1;
    const int RZ = d->dim == 3 ? R : 0;
    double s = 0.0;
    for (int kz = -RZ; kz <= RZ; ++kz)
        for (int ky = -R; ky <= R; ++ky)
            for (int kx = -R; kx <= R; ++kx) {
                const double q = d->dx * std::sqrt((double)(kx * kx + ky * ky + kz * kz)) / h;
                if (q < 2.0) {
                    const double t = 1.0 - 0.5 * q;
                    s += alpha * t * t * t * t * (1.0 + 2.0 * q);
                }
            }
    d->sigma0 = s;
    return SPH_OK;
}

size_t sph_scratch_bytes(const sph_desc* d, int64_t n_fluid, int64_t n_wall) {
    if (!d || n_fluid < 0 || n_wall < 0 || n_fluid > max_particles(d) || n_wall > max_particles(d)) return 0;
    return layout(d, n_fluid, n_wall, nullptr).bytes;
}

#define SPH_ENTRY_CHECKS()                 \
    int rc_ = check_desc(d);               \
    if (rc_) return rc_;                   \
    rc_ = check_buf(d, b);                 \
    if (rc_) return rc_;                   \
    hipStream_t st = (hipStream_t)stream;

int sph_init(const sph_desc* d, sph_buffers* b, const double* fpos, const double* fvel,
             const double* frho, const double* wpos, void* stream) {
    SPH_ENTRY_CHECKS();
    if (b->n_fluid > 0 && (!fpos || !fvel || !frho)) return SPH_ERR_ARG;
    if (b->n_wall > 0 && !wpos) return SPH_ERR_ARG;
    return SPH_DISPATCH(init_t, d, b, fpos, fvel, frho, wpos, st);
}

int sph_build_cells(const sph_desc* d, sph_buffers* b, void* stream) {
    SPH_ENTRY_CHECKS();
    return SPH_DISPATCH(build_cells_t, d, b, st);
}

int sph_density(const sph_desc* d, sph_buffers* b, void* stream) {
    SPH_ENTRY_CHECKS();
    return SPH_DISPATCH(density_t, d, b, st);
}

int sph_wall_bc(const sph_desc* d, sph_buffers* b, void* stream) {
    SPH_ENTRY_CHECKS();
    return SPH_DISPATCH(wall_bc_t, d, b, st);
}

int sph_forces(const sph_desc* d, sph_buffers* b, unsigned which, void* stream) {
    SPH_ENTRY_CHECKS();
    const unsigned kind = which & (SPH_CONTINUITY | SPH_MOMENTUM);
    if (kind != SPH_CONTINUITY && kind != SPH_MOMENTUM) return SPH_ERR_ARG;
    if ((which & SPH_NO_KICK) && kind != SPH_MOMENTUM) return SPH_ERR_ARG;
    if (which & ~(SPH_CONTINUITY | SPH_MOMENTUM | SPH_NO_KICK)) return SPH_ERR_ARG;
    return SPH_DISPATCH(forces_t, d, b, which, st);
}

int sph_step(const sph_desc* d, sph_buffers* b, int nsteps, void* stream) {
    SPH_ENTRY_CHECKS();
    if (nsteps < 0) return SPH_ERR_ARG;
    return SPH_DISPATCH(step_t, d, b, nsteps, st);
}

int sph_step_frame(const sph_desc* d, sph_buffers* b, void* sigma_cur, sph_frame* next, void* stream) {
    SPH_ENTRY_CHECKS();
    if (!next) return SPH_ERR_ARG;
    if (b->n_fluid > 0 && (!sigma_cur || !next->key || !next->pid || !next->off || !next->fstart ||
                           !next->vh || !next->rt || !next->rho))
        return SPH_ERR_ARG;
    if (b->n_wall > 0 && !next->pw) return SPH_ERR_ARG;
    return SPH_DISPATCH(step_frame_t, d, b, sigma_cur, next, st);
}

int sph_diag(const sph_desc* d, sph_buffers* b, void* stream) {
    SPH_ENTRY_CHECKS();
    return SPH_DISPATCH(diag_t, d, b, st);
}

int sph_diag_noalloc(const sph_desc* d, sph_buffers* b, void* stream) {
    int rc = check_desc(d);
    if (rc) return rc;
    rc = check_state(d, b);  // b->scratch is not read
    if (rc) return rc;
    if (b->n_fluid > SPH_DIAG_NOALLOC_MAX_FLUID) return SPH_ERR_CAPACITY;
    void* part = nullptr;
    rc = static_scratch(&part);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    return SPH_DISPATCH(diag_static_t, d, b, (double*)part, st);
}

int sph_export(const sph_desc* d, const sph_buffers* b, double* pos, double* vel, double* rho,
               double* acc, void* stream) {
    SPH_ENTRY_CHECKS();
    return SPH_DISPATCH(export_t, d, b, pos, vel, rho, acc, st);
}

int sph_export_walls(const sph_desc* d, const sph_buffers* b, double* pw, double* nrm, double* pos,
                     void* stream) {
    SPH_ENTRY_CHECKS();
    return SPH_DISPATCH(export_walls_t, d, b, pw, nrm, pos, st);
}

int sph_neighbours(const sph_desc* d, const sph_buffers* b, int which, const int64_t* offset,
                   int32_t* count, int32_t* list, int64_t list_len, void* stream) {
    SPH_ENTRY_CHECKS();
    if (which != 0 && which != 1) return SPH_ERR_ARG;
    if (!count || (list && (!offset || list_len < 0))) return SPH_ERR_ARG;
    return SPH_DISPATCH(neighbours_t, d, b, which, offset, count, list, list_len, st);
}

const char* sph_strerror(int code) {
    switch (code) {
        case SPH_OK: return "ok";
        case SPH_ERR_ARG: return "invalid argument (null pointer, size or flag)";
        case SPH_ERR_CONFIG: return "invalid configuration (dim, precision, grid, or dt above the CFL bound)";
        case SPH_ERR_LAUNCH: return "a HIP call failed (kernel launch or device symbol lookup)";
        case SPH_ERR_CAPACITY: return "more fluid particles than the fixed device workspace of sph_diag_noalloc holds";
        default: return "unknown error";
    }
}

}  // extern "C"
