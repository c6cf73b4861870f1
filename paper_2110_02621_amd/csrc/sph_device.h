// sph_device.h -- device-side building blocks of the gfx950 SPH hot path:
// run constants, XCD-aware block numbering, the cell+offset pair distance,
// the 27-cell (3-D) / 9-cell (2-D) neighbour walk and the Wendland kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sph {

constexpr int kBlock = 256;  // threads per block for per-particle kernels (4 wave64)
constexpr int kXcd = 8;      // MI355X: 8 accelerator complex dies, 32 CUs each

// Run constants in the working precision T, passed by value to every kernel.
template <typename T>
struct Par {
    int nx, ny, nz;  // cells per axis
    int penalty;     // 1: penalty force on fluid-wall pairs
    T L;             // cell edge L_c (>= the support radius 2h)
    T rc2;           // (2h)^2 rounded to T: pair iff r^2 < rc2
    T hinv;          // 1/h
    T alpha;         // Wendland normalisation a_d
    T gfac;          // -5 a_d / h^2, so that W'(r)/r = gfac (1 - q/2)^3
    T m;             // particle mass rho0 dx^d (fluid and walls)
    T vol;           // dx^d, wall volume in Eq. (16)
    T rho0, c, c2, cinv, inv_c2;
    T mu2;           // 2 mu
    T eta2;          // 0.01 h^2 (viscous regulariser)
    T gamma_p;
    T two_over_dx;   // 2/dx of Eq. (15)
    T g[3];          // body force
    T gw[3];         // g - a_w of Eq. (12)
    T dt, half_dt;
    T sigma0;        // reference number density of Eq. (17)
    T rho0_over_sigma0;
    T psi_min;       // normals with |Psi| <= psi_min are set to 0
};

// Blocks are handed to the 8 XCDs round-robin (block b runs on XCD b % 8).
// Renumber so that each XCD works on one contiguous range of particles: the
// neighbour data a block reads then stays in that XCD's own L2.
__device__ __forceinline__ int logical_block() {
    const int nb = gridDim.x, b = blockIdx.x;
    const int q = nb / kXcd, r = nb % kXcd;
    const int x = b % kXcd, k = b / kXcd;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}

__device__ __forceinline__ int64_t global_index() {
    return (int64_t)logical_block() * blockDim.x + threadIdx.x;
}

// Precision-generic math with explicit float and double forms (the float
// forms map to single gfx950 instructions).
__device__ __forceinline__ float root(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double root(double x) { return __builtin_sqrt(x); }
__device__ __forceinline__ float absv(float x) { return __builtin_fabsf(x); }
__device__ __forceinline__ double absv(double x) { return __builtin_fabs(x); }
__device__ __forceinline__ float minv(float a, float b) { return __builtin_fminf(a, b); }
__device__ __forceinline__ double minv(double a, double b) { return __builtin_fmin(a, b); }
__device__ __forceinline__ float maxv(float a, float b) { return __builtin_fmaxf(a, b); }
__device__ __forceinline__ double maxv(double a, double b) { return __builtin_fmax(a, b); }
__device__ __forceinline__ float floorv(float x) { return __builtin_floorf(x); }
__device__ __forceinline__ double floorv(double x) { return __builtin_floor(x); }
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq(double x) { return 1.0 / sqrt(x); }

// Relative vector r_i - r_j from cell + offset: with s = c_j - c_i per axis,
// d = (o_i - o_j) - s L, every operation rounded on its own (no fused
// multiply-add), and r^2 = (d0 d0 + d1 d1) + d2 d2.  The pair test r^2 < rc2
// is thereby fully defined in T.
template <typename T, int D>
__device__ __forceinline__ T rel2(const T oi[3], T ox, T oy, T oz, T sx, T sy, T sz, T d[3]) {
#pragma clang fp contract(off)
    d[0] = (oi[0] - ox) - sx;
    d[1] = (oi[1] - oy) - sy;
    T r2 = d[0] * d[0] + d[1] * d[1];
    if (D == 3) {
        d[2] = (oi[2] - oz) - sz;
        r2 = r2 + d[2] * d[2];
    } else {
        d[2] = T(0);
    }
    return r2;
}

// Cell coordinates of a linear key = cx + nx (cy + ny cz).
template <typename T>
__device__ __forceinline__ void cell_of(const Par<T>& P, int key, int c[3]) {
    c[0] = key % P.nx;
    const int t = key / P.nx;
    c[1] = t % P.ny;
    c[2] = t / P.ny;
}

// Neighbour list entries: index j in the low 26 bits, the cell shift
// c_j - c_i + 1 per axis in two bits each above it.
constexpr uint32_t kIdxBits = 26;
constexpr uint32_t kIdxMask = (1u << kIdxBits) - 1u;

__device__ __forceinline__ uint32_t shift_code(int sx, int sy, int sz) {
    return (uint32_t)((sx + 1) | ((sy + 1) << 2) | ((sz + 1) << 4)) << kIdxBits;
}

// Visit every particle j of a cell-sorted set with |r_i - r_j|^2 < rc2,
// for a query point in cell c with offset oi.  The x-neighbours of a cell
// are adjacent in key order, so each (y, z) row of 3 cells is one
// contiguous index range; the cell of j inside the row follows from the
// row's cell starts.  f(j, d, r2, code) receives d = r_i - r_j and the
// shift code of the pair.
template <typename T, int D, typename F>
__device__ __forceinline__ void for_neighbours(const Par<T>& P, const int32_t* __restrict__ start,
                                               const T* __restrict__ o0, const T* __restrict__ o1,
                                               const T* __restrict__ o2, const int c[3],
                                               const T oi[3], F&& f) {
    const int zlo = D == 3 ? max(c[2] - 1, 0) : 0;
    const int zhi = D == 3 ? min(c[2] + 1, P.nz - 1) : 0;
    const int ylo = max(c[1] - 1, 0), yhi = min(c[1] + 1, P.ny - 1);
    const int xlo = max(c[0] - 1, 0), xhi = min(c[0] + 1, P.nx - 1);
    for (int z = zlo; z <= zhi; ++z) {
        const T sz = T(z - c[2]) * P.L;
        for (int y = ylo; y <= yhi; ++y) {
            const T sy = T(y - c[1]) * P.L;
            const uint32_t cyz = shift_code(0, y - c[1], z - c[2]) & ~(3u << kIdxBits);
            const int row = P.nx * (y + P.ny * z);
            const int j0 = start[row + xlo];
            const int jm = start[row + c[0]];
            const int jp = start[row + c[0] + 1];
            const int j1 = start[row + xhi + 1];
            for (int j = j0; j < j1; ++j) {
                const int ix = j < jm ? -1 : (j < jp ? 0 : 1);
                const T sx = T(ix) * P.L;
                T d[3];
                const T r2 = rel2<T, D>(oi, o0[j], o1[j], D == 3 ? o2[j] : T(0), sx, sy, sz, d);
                if (r2 < P.rc2) f(j, d, r2, cyz | ((uint32_t)(ix + 1) << kIdxBits));
            }
        }
    }
}

// Neighbour list of one query particle: entry k at list[k * stride + i]
// (interleaved: a wave reads one entry of 64 particles in one coalesced
// access).  The distance is recomputed exactly as in the cell walk, so a
// sweep over the list sees bit-identical d and r^2, in the same order.
struct NbrList {
    const uint32_t* list;  // null: no list, walk the cells
    const int32_t* count;
    int64_t stride;
    int cap;
};

template <typename T, int D, typename F>
__device__ __forceinline__ void for_list(const Par<T>& P, const uint32_t* __restrict__ list,
                                         int64_t stride, int64_t i, int n,
                                         const T* __restrict__ o0, const T* __restrict__ o1,
                                         const T* __restrict__ o2, const T oi[3], F&& f) {
    for (int k = 0; k < n; ++k) {
        const uint32_t e = list[(int64_t)k * stride + i];
        const int j = (int)(e & kIdxMask);
        const T sx = T((int)((e >> 26) & 3u) - 1) * P.L;
        const T sy = T((int)((e >> 28) & 3u) - 1) * P.L;
        const T sz = T((int)((e >> 30) & 3u) - 1) * P.L;
        T d[3];
        const T r2 = rel2<T, D>(oi, o0[j], o1[j], D == 3 ? o2[j] : T(0), sx, sy, sz, d);
        f(j, d, r2, e & ~kIdxMask);
    }
}

// The neighbours of query i: from its list when one exists and did not
// overflow, else by walking the cells.
template <typename T, int D, typename F>
__device__ __forceinline__ void visit(const Par<T>& P, const NbrList& NL, int64_t i,
                                      const int32_t* __restrict__ start, const T* __restrict__ o0,
                                      const T* __restrict__ o1, const T* __restrict__ o2,
                                      const int c[3], const T oi[3], F&& f) {
    if (NL.list) {
        const int n = NL.count[i];
        if (n <= NL.cap) {
            for_list<T, D>(P, NL.list, NL.stride, i, n, o0, o1, o2, oi, f);
            return;
        }
    }
    for_neighbours<T, D>(P, start, o0, o1, o2, c, oi, f);
}

// Quintic Wendland C2 (kappa = 2) at r: q = r/h, t = 1 - q/2,
// W = a_d t^4 (1 + 2q) and W'(r)/r = -5 a_d t^3 / h^2.
template <typename T>
__device__ __forceinline__ T wendland_W(const Par<T>& P, T r) {
    const T q = r * P.hinv;
    const T t = T(1) - T(0.5) * q;
    const T t2 = t * t;
    return P.alpha * (t2 * t2) * (T(1) + T(2) * q);
}

template <typename T>
__device__ __forceinline__ T wendland_F(const Par<T>& P, T r) {
    const T t = T(1) - T(0.5) * r * P.hinv;
    return P.gfac * (t * t * t);
}

}  // namespace sph
