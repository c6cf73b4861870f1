// sph_device.h -- device-side building blocks of the gfx950 SPH hot path:
// run constants, XCD-aware block numbering, the cell+offset pair distance,
// the 27-cell (3-D) / 9-cell (2-D) neighbour walk, neighbour bitmasks and
// the Wendland kernel.
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
    int two_phase;   // 1: particles with initial index >= n_heavy are the light phase
    int n_heavy;
    T rho0L;         // light-phase reference density
    T rho0L_over_sigma0;
    T fk[3];         // uniform velocity added by this call's kick (moving tank; else 0)
    int cross_phase; // two phases: light particles see heavy ones as moving wall dummies
};

// Reference density of the particle with initial index pid.
template <typename T>
__device__ __forceinline__ T ref_density(const Par<T>& P, int pid) {
    return (P.two_phase && pid >= P.n_heavy) ? P.rho0L : P.rho0;
}

// Blocks are handed to the 8 XCDs round-robin (block b runs on XCD b % 8).
// C = 0: renumber so that each XCD works on one contiguous range of
// particles, so the neighbour data a block reads stays in that XCD's own
// L2 (the pair sweeps).  C > 0: each XCD takes chunks of C consecutive
// blocks in turn (blocks past the last full round keep their number), which
// keeps a chunk's neighbour rows in one L2 while spreading regions of
// uneven work, such as the particles next to the tank floor that come first
// in cell order, over all XCDs (the mask builders, the wall pressure and
// the streaming kernels).
template <int C = 0>
__device__ __forceinline__ int logical_block() {
    const int nb = gridDim.x, b = blockIdx.x;
    const int x = b % kXcd, k = b / kXcd;
    if (C == 0) {
        const int q = nb / kXcd, r = nb % kXcd;
        return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
    }
    const int full = nb / (C * kXcd);  // complete rounds of chunks
    return k / C < full ? ((k / C) * kXcd + x) * C + (k % C) : b;
}

constexpr int kChunk = 64;  // blocks per chunk of the chunked numbering

template <int C = 0>
__device__ __forceinline__ int64_t global_index() {
    return (int64_t)logical_block<C>() * blockDim.x + threadIdx.x;
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

// Element j of a device array through a 32-bit byte offset from the array's
// (wave-uniform) base, so the load takes the scalar-base addressing form and
// needs no 64-bit address arithmetic per lane.  The entry points refuse
// particle counts whose record arrays would reach 4 GiB (2^28 particles in
// FP32, 2^27 in FP64), so the offset never wraps.
template <typename T>
__device__ __forceinline__ T ldg(const T* __restrict__ p, int j) {
    return *(const T*)((const char*)p + (uint32_t)j * (uint32_t)sizeof(T));
}

// x shift of candidate j of a row: -L left of the query's cell [jm, jp),
// 0 inside, +L right of it (the same values as T(ix) * L).
template <typename T>
__device__ __forceinline__ T row_shift(int j, int jm, int jp, T L) {
    return j < jm ? -L : (j < jp ? T(0) : L);
}

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

// Cell shift code of a pair: c_j - c_i + 1 per axis in two bits each,
// above bit 26 (passed to the neighbour callbacks).
constexpr uint32_t kIdxBits = 26;

__device__ __forceinline__ uint32_t shift_code(int sx, int sy, int sz) {
    return (uint32_t)((sx + 1) | ((sy + 1) << 2) | ((sz + 1) << 4)) << kIdxBits;
}

// The neighbour stencil is the 3 (2-D) or 9 (3-D) (y, z) rows of three
// x-adjacent cells around the query's cell, numbered (dz + 1) * 3 + (dy + 1).
// A row is skipped when its y/z gap alone puts all of it beyond the support,
// its left or right cell when the x gap does.  The margin (1 + 1e-5) on rc2
// keeps every skip conservative against rounding, so the pair set (decided
// by the exact r^2 < rc2 test) is unchanged.
constexpr int kMaskWords = 2;  // 128 candidates per row
constexpr double kSkipMargin = 1.0 + 1e-5;

template <typename T>
__device__ __forceinline__ T gap(int dcell, T o, T L) {
    return dcell < 0 ? o : (dcell > 0 ? L - o : T(0));
}

template <int D>
__device__ __forceinline__ int stencil_row(int dy, int dz) {
    return D == 3 ? (dz + 1) * 3 + (dy + 1) : (dy + 1);
}

// Order in which every neighbour loop visits the stencil rows: each row
// followed by its mirror image (dy, dz) -> (-dy, -dz), the centre row last
// (3-D: 0, 8, 1, 7, 2, 6, 3, 5, 4).  A particle's pair counts in a row and
// in its mirror vary in opposite directions with its place in the cell, so
// a loop over the two together keeps the lanes of a wave evenly loaded.
template <int D>
constexpr int kRows = D == 3 ? 9 : 3;

template <int D>
__device__ __forceinline__ int row_at(int k) {
    constexpr int last = kRows<D> - 1;
    return k == last ? last / 2 : ((k & 1) ? last - (k >> 1) : (k >> 1));
}

// (y, z) of stencil row r around the cell row (cy, cz); false when outside
// the grid.
template <typename T, int D>
__device__ __forceinline__ bool row_cell(const Par<T>& P, int r, int cy, int cz, int& y, int& z) {
    y = cy + r % 3 - 1;
    z = D == 3 ? cz + r / 3 - 1 : 0;
    return y >= 0 && y < P.ny && z >= 0 && z < (D == 3 ? P.nz : 1);
}

// One stencil row as the walk, the mask builder and the mask sweep all see
// it: cell starts and the (possibly trimmed) candidate range.
struct Row {
    int base;    // start of the row's full 3-cell range (mask bit 0)
    int jm, jp;  // start and end of the query's own cell in the row
    int j0, j1;  // candidate range after trimming
    int r;       // stencil row number
    uint32_t cyz;
};

// Row (y, z) of query (c, oi): false when the row is skipped (its y/z gap
// alone reaches past the support, or no candidate is left after trimming
// its left and right cells).  Contraction is off so that every kernel that
// inlines this (the mask builder and all sweeps) takes the same decisions.
template <typename T, int D>
__device__ __forceinline__ bool row_of(const Par<T>& P, const int32_t* __restrict__ start, const int c[3],
                                       const T oi[3], int y, int z, Row& R) {
#pragma clang fp contract(off)
    const T reach = P.rc2 * T(kSkipMargin);
    const T gz = D == 3 ? gap(z - c[2], oi[2], P.L) : T(0);
    const T gy = gap(y - c[1], oi[1], P.L);
    const T g2 = gy * gy + gz * gz;
    if (!(g2 < reach)) return false;
    const T rx2 = reach - g2;
    const T gl = oi[0], gr = P.L - oi[0];
    const int row = P.nx * (y + P.ny * z);
    const bool left = c[0] > 0 && gl * gl < rx2;
    const bool right = c[0] < P.nx - 1 && gr * gr < rx2;
    R.base = start[row + max(c[0] - 1, 0)];
    R.jm = start[row + c[0]];
    R.jp = start[row + c[0] + 1];
    R.j0 = left ? R.base : R.jm;
    R.j1 = right ? start[row + c[0] + 2] : R.jp;
    if (R.j0 >= R.j1) return false;  // no candidates: no mask word is written or read
    R.r = stencil_row<D>(y - c[1], z - c[2]);
    R.cyz = shift_code(0, y - c[1], z - c[2]) & ~(3u << kIdxBits);
    return true;
}

// Iterate the rows of query (c, oi) in the order of row_at; g(row, sy, sz)
// is called per row kept.
template <typename T, int D, typename G>
__device__ __forceinline__ void for_rows(const Par<T>& P, const int32_t* __restrict__ start,
                                         const int c[3], const T oi[3], G&& g) {
    for (int k = 0; k < kRows<D>; ++k) {
        int y, z;
        if (!row_cell<T, D>(P, row_at<D>(k), c[1], c[2], y, z)) continue;
        Row R;
        if (!row_of<T, D>(P, start, c, oi, y, z, R)) continue;
        g(R, T(y - c[1]) * P.L, T(z - c[2]) * P.L);
    }
}

// Packed per-particle record: three components and one extra value in one
// 16-byte (FP32) or 32-byte (FP64) load.  The sweeps gather neighbour data
// through these records: the texture addresser handles a gather by lanes,
// so one record load costs what one scalar load does and brings four.
template <typename T>
struct alignas(4 * sizeof(T)) Rec {
    T x, y, z, w;
};

template <typename T>
__device__ __forceinline__ Rec<T> ld4(const Rec<T>* __restrict__ p, int j) {
    return *(const Rec<T>*)((const char*)p + (uint32_t)j * (uint32_t)sizeof(Rec<T>));
}

// Neighbour position sources: separate component arrays (w = 0), or
// packed records (x, y, z = offset; w = the value stored with it).
template <typename T, int D>
struct SoaSrc {
    const T *x, *y, *z;
    __device__ __forceinline__ Rec<T> operator()(int j) const {
        Rec<T> q;
        q.x = ldg(x, j);
        q.y = ldg(y, j);
        q.z = D == 3 ? ldg(z, j) : T(0);
        q.w = T(0);
        return q;
    }
};

template <typename T>
struct PackSrc {
    const Rec<T>* p;
    __device__ __forceinline__ Rec<T> operator()(int j) const { return ld4(p, j); }
};

// Visit every particle j of a cell-sorted set with |r_i - r_j|^2 < rc2,
// for a query point in cell c with offset oi.  The x-neighbours of a cell
// are adjacent in key order, so each (y, z) row of 3 cells is one
// contiguous index range; the cell of j inside the row follows from the
// row's cell starts.  f(j, d, r2, code, q) receives d = r_i - r_j, the
// shift code of the pair and j's record from the source.  Pairs come row
// by row, the rows in the order of row_at, each in ascending j.
template <typename T, int D, typename S, typename F>
__device__ __forceinline__ void walk_src(const Par<T>& P, const int32_t* __restrict__ start, const S& src,
                                         const int c[3], const T oi[3], F&& f) {
    for_rows<T, D>(P, start, c, oi, [&](const Row& R, T sy, T sz) {
        for (int j = R.j0; j < R.j1; ++j) {
            const int ix = j < R.jm ? -1 : (j < R.jp ? 0 : 1);
            const Rec<T> q = src(j);
            T d[3];
            const T r2 = rel2<T, D>(oi, q.x, q.y, q.z, row_shift(j, R.jm, R.jp, P.L), sy, sz, d);
            if (r2 < P.rc2) f(j, d, r2, R.cyz | ((uint32_t)(ix + 1) << kIdxBits), q);
        }
    });
}

template <typename T, int D, typename F>
__device__ __forceinline__ void for_neighbours(const Par<T>& P, const int32_t* __restrict__ start,
                                               const T* __restrict__ o0, const T* __restrict__ o1,
                                               const T* __restrict__ o2, const int c[3],
                                               const T oi[3], F&& f) {
    walk_src<T, D>(P, start, SoaSrc<T, D>{o0, o1, o2}, c, oi,
                   [&](int j, const T* d, T r2, uint32_t code, const Rec<T>&) { f(j, d, r2, code); });
}

// Neighbour masks of one set: for query q and stencil row r, the words
// mask[(r * kMaskWords + w) * n + q] hold one bit per candidate of the
// row's full 3-cell index range: bit b of word w marks candidate
// base + 64 w + b as a pair.  count[q] is the number of pairs, or -1 when a
// row had more than 128 candidates (that query walks the cells instead).
// Rows without candidates, and the second word of rows of at most 64
// candidates, are neither written nor read.
// Storage is interleaved across queries: a wave reads or writes one word
// of 64 queries in one coalesced access.
struct NbrMask {
    const uint64_t* mask;  // null: no masks, walk the cells
    const int32_t* count;
    int64_t n;
};

// Pair bits of candidates [ja, jb) of one cell of a row into one mask word
// whose bit 0 is candidate wbase (jb - wbase <= 64): bit j - wbase is set
// when j is a neighbour.  sx is the cell's x shift (what row_shift gives for
// every j of the cell), so the distance is the same arithmetic as the
// walk's.  get(j) returns j's position record.  The candidates are tested
// in chunks of up to 32, each from its last candidate down, shifting the
// results into a 32-bit word that is then placed at the chunk's offset.
template <typename T, int D, typename Get>
__device__ __forceinline__ uint64_t cell_bits(const Par<T>& P, int ja, int jb, int wbase, T sx, const T oi[3],
                                              T sy, T sz, Get&& get) {
    uint64_t m = 0;
    for (int c0 = ja; c0 < jb; c0 += 32) {
        const int c1 = jb - c0 < 32 ? jb : c0 + 32;
        uint32_t w = 0;
        int j = c1 - 1;
        for (; j > c0 + 2; j -= 4) {  // four at a time: bit j - c0 of w once the chunk is done
            const Rec<T> q0 = get(j - 3), q1 = get(j - 2), q2 = get(j - 1), q3 = get(j);
            T d[3];
            const T r0 = rel2<T, D>(oi, q0.x, q0.y, q0.z, sx, sy, sz, d);
            const T r1 = rel2<T, D>(oi, q1.x, q1.y, q1.z, sx, sy, sz, d);
            const T r2 = rel2<T, D>(oi, q2.x, q2.y, q2.z, sx, sy, sz, d);
            const T r3 = rel2<T, D>(oi, q3.x, q3.y, q3.z, sx, sy, sz, d);
            w = (w << 4) | (r3 < P.rc2 ? 8u : 0u) | (r2 < P.rc2 ? 4u : 0u) | (r1 < P.rc2 ? 2u : 0u) |
                (r0 < P.rc2 ? 1u : 0u);
        }
        for (; j >= c0; --j) {
            const Rec<T> q = get(j);
            T d[3];
            const T r2 = rel2<T, D>(oi, q.x, q.y, q.z, sx, sy, sz, d);
            w = (w << 1) | (r2 < P.rc2 ? 1u : 0u);
        }
        m |= (uint64_t)w << (c0 - wbase);
    }
    return m;
}

// Candidates [ja, jb) of one cell of row R into the row's two words.
template <typename T, int D, typename Get>
__device__ __forceinline__ void cell_words(const Par<T>& P, const Row& R, int ja, int jb, T sx, const T oi[3],
                                           T sy, T sz, Get&& get, uint64_t& m0, uint64_t& m1) {
    const int split = R.base + 64;
    m0 |= cell_bits<T, D>(P, ja, jb < split ? jb : split, R.base, sx, oi, sy, sz, get);
    if (jb > split)
        m1 |= cell_bits<T, D>(P, ja > split ? ja : split, jb < split + 64 ? jb : split + 64, split, sx, oi, sy,
                              sz, get);
}

// Both words of row R, cell by cell (left, own, right), each with its
// constant x shift; candidates past base + 128 are not recorded (the caller
// flags the row as overflowing).
template <typename T, int D, typename Get>
__device__ __forceinline__ void row_words(const Par<T>& P, const Row& R, const T oi[3], T sy, T sz, Get&& get,
                                          uint64_t& m0, uint64_t& m1) {
    m0 = 0;
    m1 = 0;
    cell_words<T, D>(P, R, R.j0, R.jm, -P.L, oi, sy, sz, get, m0, m1);
    cell_words<T, D>(P, R, R.jm, R.jp, T(0), oi, sy, sz, get, m0, m1);
    cell_words<T, D>(P, R, R.jp, R.j1, P.L, oi, sy, sz, get, m0, m1);
}

// Build the masks of query i (rows kept by the walk only).  Returns the
// pair count, or -1 on a row with more than 128 candidates.
template <typename T, int D, typename S>
__device__ __forceinline__ int build_mask(const Par<T>& P, const int32_t* __restrict__ start, const S& src,
                                          const int c[3], const T oi[3], uint64_t* __restrict__ mask,
                                          int64_t n, int64_t i) {
    int count = 0;
    bool over = false;
    for_rows<T, D>(P, start, c, oi, [&](const Row& R, T sy, T sz) {
        uint64_t m0, m1;
        if (R.j1 - R.base > 64 * kMaskWords) over = true;
        row_words<T, D>(P, R, oi, sy, sz, src, m0, m1);
        count += __builtin_popcountll(m0) + __builtin_popcountll(m1);
        mask[(int64_t)(R.r * kMaskWords + 0) * n + i] = m0;
        if (R.j1 - R.base > 64) mask[(int64_t)(R.r * kMaskWords + 1) * n + i] = m1;
    });
    return over ? -1 : count;
}

// Visit the pairs recorded in the masks of query i: same rows and the
// same ascending order as the walk, so sums are bit-identical to it.  All
// lanes of a wave sweep one row at a time, so their gathers fall into the
// same few cells.
template <typename T, int D, typename S, typename F>
__device__ __forceinline__ void mask_src(const Par<T>& P, const int32_t* __restrict__ start, const S& src,
                                         const int c[3], const T oi[3], const uint64_t* __restrict__ mask,
                                         int64_t n, int64_t i, F&& f) {
    for_rows<T, D>(P, start, c, oi, [&](const Row& R, T sy, T sz) {
        // the second word exists only for rows of more than 64 candidates
        const uint64_t m[kMaskWords] = {
            mask[(int64_t)(R.r * kMaskWords + 0) * n + i],
            R.j1 - R.base > 64 ? mask[(int64_t)(R.r * kMaskWords + 1) * n + i] : 0ull};
#pragma unroll
        for (int w = 0; w < kMaskWords; ++w) {
            uint64_t bits = m[w];
            while (bits) {
                const int j = R.base + 64 * w + __builtin_ctzll(bits);
                bits &= bits - 1;
                const int ix = j < R.jm ? -1 : (j < R.jp ? 0 : 1);
                const Rec<T> q = src(j);
                T d[3];
                const T r2 = rel2<T, D>(oi, q.x, q.y, q.z, row_shift(j, R.jm, R.jp, P.L), sy, sz, d);
                f(j, d, r2, R.cyz | ((uint32_t)(ix + 1) << kIdxBits), q);
            }
        }
    });
}

// Pointer into LDS (address space 3): reads through it compile to ds_read,
// not to flat loads that would take the vector-memory path.
#define SPH_LDS __attribute__((address_space(3)))

template <typename T>
using Vec4 = T __attribute__((ext_vector_type(4)));

template <typename T>
__device__ __forceinline__ void lds_put(SPH_LDS Rec<T>* p, int k, const Rec<T>& v) {
    *(SPH_LDS Vec4<T>*)((SPH_LDS char*)p + k * (int)sizeof(Rec<T>)) = Vec4<T>{v.x, v.y, v.z, v.w};
}

template <typename T>
__device__ __forceinline__ Rec<T> lds_get(const SPH_LDS Rec<T>* p, int k) {
    const Vec4<T> t = *(const SPH_LDS Vec4<T>*)((const SPH_LDS char*)p + k * (int)sizeof(Rec<T>));
    return Rec<T>{t.x, t.y, t.z, t.w};
}

// Barrier for data that the lanes of one wave exchange through LDS.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Cells spanned by the wave whose first particle is ib (consecutive sorted
// particles): when all of them lie in one (y, z) row of cells (one_row), the
// candidates of each stencil row of every lane lie in one index range,
// [start of cell cx0 - 1, end of cell cx1 + 1) of that row.
struct WaveSpan {
    bool one_row;
    int cy, cz, cx0, cx1;
};

template <typename T>
__device__ __forceinline__ WaveSpan span_of(const Par<T>& P, const int32_t* __restrict__ key, int64_t first,
                                            int64_t last) {
    const int k0 = key[first], k1 = key[last];
    const int r0 = k0 / P.nx, r1 = k1 / P.nx;
    WaveSpan S;
    S.one_row = r0 == r1;
    S.cx0 = k0 - r0 * P.nx;
    S.cx1 = k1 - r1 * P.nx;
    S.cy = r0 % P.ny;
    S.cz = r0 / P.ny;
    return S;
}

template <typename T>
__device__ __forceinline__ WaveSpan wave_span(const Par<T>& P, const int32_t* __restrict__ key, int64_t ib,
                                              int64_t n) {
    return span_of(P, key, ib, ib + 63 < n ? ib + 63 : n - 1);
}

// Visit the set bits of one mask word of row R (candidates wbase + bit) in
// ascending order; get(j, q, u) loads j's position and velocity records.
template <typename T, int D, typename Get, typename F>
__device__ __forceinline__ void bits_loop(const Par<T>& P, const Row& R, int wbase, uint64_t bits,
                                          const T oi[3], T sy, T sz, Get&& get, F&& f) {
    while (bits) {
        const int j = wbase + __builtin_ctzll(bits);
        bits &= bits - 1;
        const int ix = j < R.jm ? -1 : (j < R.jp ? 0 : 1);
        Rec<T> q, u;
        get(j, q, u);
        T d[3];
        const T r2 = rel2<T, D>(oi, q.x, q.y, q.z, row_shift(j, R.jm, R.jp, P.L), sy, sz, d);
        f(j, d, r2, R.cyz | ((uint32_t)(ix + 1) << kIdxBits), q, u);
    }
}

// A kept row of a masked sweep: its (one or two) words, with the records
// from LDS when staged (at index j - ulo) or from memory.
template <typename T, int D, typename F>
__device__ __forceinline__ void masked_row(const Par<T>& P, const Row& R, const uint64_t* __restrict__ mask,
                                           int64_t n, int64_t i, const T oi[3], T sy, T sz, bool staged,
                                           const SPH_LDS Rec<T>* sp, const SPH_LDS Rec<T>* sv, int ulo,
                                           const Rec<T>* __restrict__ pk, const Rec<T>* __restrict__ vk, F&& f) {
    const uint64_t m0 = mask[(int64_t)(R.r * kMaskWords + 0) * n + i];
    const uint64_t m1 = R.j1 - R.base > 64 ? mask[(int64_t)(R.r * kMaskWords + 1) * n + i] : 0ull;
    if (staged) {
        auto get = [&](int j, Rec<T>& q, Rec<T>& u) {
            q = lds_get(sp, j - ulo);
            u = lds_get(sv, j - ulo);
        };
        bits_loop<T, D>(P, R, R.base, m0, oi, sy, sz, get, f);
        bits_loop<T, D>(P, R, R.base + 64, m1, oi, sy, sz, get, f);
    } else {
        auto get = [&](int j, Rec<T>& q, Rec<T>& u) {
            q = ld4(pk, j);
            u = ld4(vk, j);
        };
        bits_loop<T, D>(P, R, R.base, m0, oi, sy, sz, get, f);
        bits_loop<T, D>(P, R, R.base + 64, m1, oi, sy, sz, get, f);
    }
}

// Masked sweep with LDS-staged neighbour rows, for a wave in one row of
// cells (WaveSpan::one_row): per stencil row the wave loads the row's index
// range once, coalesced, into LDS (positions sp, velocities sv; at most CAP
// records, else the row is gathered from memory), and each lane reads its
// masked neighbours from there.  Lanes with on = false only help staging.
// Pairs come in the order of mask_src, so sums are bit-identical to it.
// f(j, d, r2, code, q, u) gets j's position record q and velocity record u.
template <typename T, int D, int CAP, typename F>
__device__ __forceinline__ void mask_staged(const Par<T>& P, const int32_t* __restrict__ start,
                                            const Rec<T>* __restrict__ pk, const Rec<T>* __restrict__ vk,
                                            SPH_LDS Rec<T>* sp, SPH_LDS Rec<T>* sv, const WaveSpan& S, bool on,
                                            const int c[3], const T oi[3], const uint64_t* __restrict__ mask,
                                            int64_t n, int64_t i, F&& f) {
    const int lane = threadIdx.x & 63;
    for (int k = 0; k < kRows<D>; ++k) {
        int y, z;
        if (!row_cell<T, D>(P, row_at<D>(k), S.cy, S.cz, y, z)) continue;
        Row R;
        const bool kept = on && row_of<T, D>(P, start, c, oi, y, z, R);
        if (!__any(kept)) continue;
        const int row = P.nx * (y + P.ny * z);
        const int ulo = start[row + max(S.cx0 - 1, 0)];
        const int uhi = start[row + min(S.cx1 + 1, P.nx - 1) + 1];
        const bool staged = uhi - ulo <= CAP;  // the same for every lane
        if (staged) {
            for (int t = lane; t < uhi - ulo; t += 64) {
                lds_put(sp, t, ld4(pk, ulo + t));
                lds_put(sv, t, ld4(vk, ulo + t));
            }
            wave_sync();
        }
        if (kept)
            masked_row<T, D>(P, R, mask, n, i, oi, T(y - c[1]) * P.L, T(z - c[2]) * P.L, staged, sp, sv, ulo, pk,
                             vk, f);
        if (staged) wave_sync();  // every lane is done with this row's records
    }
}

// One stencil row of a block whose particles lie in one row of cells (S):
// this thread's row (kept when it has candidates) and the block's index
// range [ulo, ulo + n) of the row, which holds every thread's candidates.
template <typename T>
struct BlockRow {
    Row R;
    bool kept;
    int ulo, n;
    T sy, sz;
};

template <typename T, int D>
__device__ __forceinline__ BlockRow<T> block_row(const Par<T>& P, const int32_t* __restrict__ start,
                                                 const WaveSpan& S, bool on, const int c[3], const T oi[3], int r) {
    BlockRow<T> B;
    B.kept = false;
    B.ulo = 0;
    B.n = 0;
    // c[1], c[2] are the block's (S.cy, S.cz): the shifts of a row and of
    // its mirror image are exact negatives of each other
    B.sy = T(r % 3 - 1) * P.L;
    B.sz = D == 3 ? T(r / 3 - 1) * P.L : T(0);
    int y, z;
    if (!row_cell<T, D>(P, r, S.cy, S.cz, y, z)) return B;  // outside the grid for the whole block
    const int row = P.nx * (y + P.ny * z);
    B.ulo = start[row + max(S.cx0 - 1, 0)];
    B.n = start[row + min(S.cx1 + 1, P.nx - 1) + 1] - B.ulo;
    B.kept = on && row_of<T, D>(P, start, c, oi, y, z, B.R);
    return B;
}

// One row on its own: staged in LDS when it fits (CAP records), else
// gathered from memory.  Every thread of the block calls it.
template <typename T, int D, int CAP, typename F>
__device__ __forceinline__ void block_single(const Par<T>& P, const BlockRow<T>& B, const Rec<T>* __restrict__ pk,
                                             const Rec<T>* __restrict__ vk, SPH_LDS Rec<T>* sp,
                                             SPH_LDS Rec<T>* sv, const T oi[3], const uint64_t* __restrict__ mask,
                                             int64_t n, int64_t i, F&& f) {
    if (!__syncthreads_or(B.kept)) return;
    const bool staged = B.n <= CAP;  // the same for every thread
    if (staged) {
        for (int t = threadIdx.x; t < B.n; t += blockDim.x) {
            lds_put(sp, t, ld4(pk, B.ulo + t));
            lds_put(sv, t, ld4(vk, B.ulo + t));
        }
        __syncthreads();
    }
    if (B.kept) masked_row<T, D>(P, B.R, mask, n, i, oi, B.sy, B.sz, staged, sp, sv, B.ulo, pk, vk, f);
    if (staged) __syncthreads();  // every thread is done with this row's records
}

// A row and its mirror image staged together (a at [0, a.n), b at
// [a.n, a.n + b.n)) and swept in one loop: each lane takes its pairs of a,
// then of b, in the order of two separate rows, so the sums are the same;
// the loop runs to the busiest lane's total over both rows instead of to
// the busiest lane of each.  A lane's state is the word it is on (bits, LDS
// index lb of its bit 0), the second word of the same row (w1), the words of
// b still to come, and the row's own-cell range and y/z shift.
template <typename T, int D, typename F>
__device__ __forceinline__ void block_pair(const Par<T>& P, const BlockRow<T>& a, const BlockRow<T>& b,
                                           const SPH_LDS Rec<T>* sp, const SPH_LDS Rec<T>* sv, const T oi[3],
                                           const uint64_t* __restrict__ mask, int64_t n, int64_t i, F&& f) {
    uint64_t bits = 0, w1 = 0, b0 = 0, b1 = 0;
    int lb = 0, ljm = 0, ljp = 0, off = 0;
    uint32_t cyz = 0;
    if (a.kept) {
        bits = mask[(int64_t)(a.R.r * kMaskWords + 0) * n + i];
        if (a.R.j1 - a.R.base > 64) w1 = mask[(int64_t)(a.R.r * kMaskWords + 1) * n + i];
        lb = a.R.base - a.ulo;
        ljm = a.R.jm - a.ulo;
        ljp = a.R.jp - a.ulo;
        off = a.ulo;
        cyz = a.R.cyz;
    }
    if (b.kept) {
        b0 = mask[(int64_t)(b.R.r * kMaskWords + 0) * n + i];
        if (b.R.j1 - b.R.base > 64) b1 = mask[(int64_t)(b.R.r * kMaskWords + 1) * n + i];
    }
    T sy = a.sy, sz = a.sz;
    bool in_a = true;
    while (true) {
        if (bits == 0) {
            if (w1 != 0) {  // second word of the same row
                bits = w1;
                w1 = 0;
                lb += 64;
            } else if (in_a && b.kept) {  // on to the mirror row
                in_a = false;
                bits = b0;
                w1 = b1;
                lb = b.R.base - b.ulo + a.n;
                ljm = b.R.jm - b.ulo + a.n;
                ljp = b.R.jp - b.ulo + a.n;
                off = b.ulo - a.n;
                cyz = b.R.cyz;
                sy = -sy;
                sz = -sz;
                if (bits == 0) {
                    bits = w1;
                    w1 = 0;
                    lb += 64;
                }
            }
            if (bits == 0) break;
        }
        const int t = lb + __builtin_ctzll(bits);
        bits &= bits - 1;
        const int ix = t < ljm ? -1 : (t < ljp ? 0 : 1);
        const Rec<T> q = lds_get(sp, t);
        const Rec<T> u = lds_get(sv, t);
        T d[3];
        const T r2 = rel2<T, D>(oi, q.x, q.y, q.z, row_shift(t, ljm, ljp, P.L), sy, sz, d);
        f(t + off, d, r2, cyz | ((uint32_t)(ix + 1) << kIdxBits), q, u);
    }
}

// Block-level form of mask_staged, for a block whose particles all lie in one
// row of cells (S spans the block): the rows go in the order of row_at, a row
// and its mirror image staged and swept together when both fit in CAP
// records, else one at a time (each staged when it fits, else gathered).
// Every thread of the block must call it.
template <typename T, int D, int CAP, typename F>
__device__ __forceinline__ void mask_block(const Par<T>& P, const int32_t* __restrict__ start,
                                           const Rec<T>* __restrict__ pk, const Rec<T>* __restrict__ vk,
                                           SPH_LDS Rec<T>* sp, SPH_LDS Rec<T>* sv, const WaveSpan& S, bool on,
                                           const int c[3], const T oi[3], const uint64_t* __restrict__ mask,
                                           int64_t n, int64_t i, F&& f) {
    constexpr int NP = kRows<D> / 2;  // mirror pairs; the centre row comes after them
    for (int g = 0; g < NP; ++g) {
        const BlockRow<T> a = block_row<T, D>(P, start, S, on, c, oi, row_at<D>(2 * g));
        const BlockRow<T> b = block_row<T, D>(P, start, S, on, c, oi, row_at<D>(2 * g + 1));
        if (!__syncthreads_or(a.kept || b.kept)) continue;
        if (a.n + b.n <= CAP) {  // the same for every thread
            for (int t = threadIdx.x; t < a.n + b.n; t += blockDim.x) {
                const int j = t < a.n ? a.ulo + t : b.ulo + (t - a.n);
                lds_put(sp, t, ld4(pk, j));
                lds_put(sv, t, ld4(vk, j));
            }
            __syncthreads();
            block_pair<T, D>(P, a, b, sp, sv, oi, mask, n, i, f);
            __syncthreads();  // every thread is done with these records
        } else {
            block_single<T, D, CAP>(P, a, pk, vk, sp, sv, oi, mask, n, i, f);
            block_single<T, D, CAP>(P, b, pk, vk, sp, sv, oi, mask, n, i, f);
        }
    }
    const BlockRow<T> m = block_row<T, D>(P, start, S, on, c, oi, row_at<D>(kRows<D> - 1));
    block_single<T, D, CAP>(P, m, pk, vk, sp, sv, oi, mask, n, i, f);
}

// Lanes of a wave sweep a row of the stencil together, so a wave runs as
// long as its busiest lane; how many neighbours a particle has in each row
// depends on where it sits in its cell across the rows (y and z).  Threads
// of a block in one row of cells therefore take the block's particles
// grouped by that position (3 bands per axis), so the lanes of each wave
// have similar per-row counts.  Returns the particle this thread sweeps.
// Which thread takes which particle changes nothing in any result.
template <typename T, int D>
__device__ __forceinline__ int64_t regroup_block(const Par<T>& P, const Rec<T>* __restrict__ pk, int64_t blk0,
                                                 int64_t nf, int* hist, int* perm) {
    const int t = threadIdx.x;
    const int64_t q = blk0 + t;
    int b = 15;  // threads past the end go last
    if (q < nf) {
        const Rec<T> me = pk[q];
        const T three = T(3) / P.L;
        const int by = min((int)(me.y * three), 2);
        const int bz = D == 3 ? min((int)(me.z * three), 2) : 0;
        b = by + 3 * bz;
    }
    if (t < 16) hist[t] = 0;
    __syncthreads();
    const int slot = atomicAdd(&hist[b], 1);
    __syncthreads();
    int off = 0;
    for (int k = 0; k < b; ++k) off += hist[k];
    perm[off + slot] = t;
    __syncthreads();
    return blk0 + perm[t];
}

// The mask builder with LDS-staged candidate rows (the union of the wave's
// row ranges, position records), for a wave in one row of cells; same
// results as build_mask.
template <typename T, int D, int CAP>
__device__ __forceinline__ int build_mask_staged(const Par<T>& P, const int32_t* __restrict__ start,
                                                 const Rec<T>* __restrict__ pk, SPH_LDS Rec<T>* sp, const WaveSpan& S,
                                                 bool on, const int c[3], const T oi[3],
                                                 uint64_t* __restrict__ mask, int64_t n, int64_t i) {
    const int lane = threadIdx.x & 63;
    const int zlo = D == 3 ? max(S.cz - 1, 0) : 0;
    const int zhi = D == 3 ? min(S.cz + 1, P.nz - 1) : 0;
    const int ylo = max(S.cy - 1, 0), yhi = min(S.cy + 1, P.ny - 1);
    int count = 0;
    bool over = false;
    for (int z = zlo; z <= zhi; ++z) {
        for (int y = ylo; y <= yhi; ++y) {
            Row R;
            const bool kept = on && row_of<T, D>(P, start, c, oi, y, z, R);
            if (!__any(kept)) continue;
            const int row = P.nx * (y + P.ny * z);
            const int ulo = start[row + max(S.cx0 - 1, 0)];
            const int uhi = start[row + min(S.cx1 + 1, P.nx - 1) + 1];
            const bool staged = uhi - ulo <= CAP;
            if (staged) {
                for (int k = lane; k < uhi - ulo; k += 64) lds_put(sp, k, ld4(pk, ulo + k));
                wave_sync();
            }
            if (kept) {
                const T sy = T(y - c[1]) * P.L, sz = T(z - c[2]) * P.L;
                uint64_t m0, m1;
                if (R.j1 - R.base > 64 * kMaskWords) over = true;
                if (staged)
                    row_words<T, D>(P, R, oi, sy, sz, [&](int j) { return lds_get(sp, j - ulo); }, m0, m1);
                else
                    row_words<T, D>(P, R, oi, sy, sz, [&](int j) { return ld4(pk, j); }, m0, m1);
                count += __builtin_popcountll(m0) + __builtin_popcountll(m1);
                mask[(int64_t)(R.r * kMaskWords + 0) * n + i] = m0;
                if (R.j1 - R.base > 64) mask[(int64_t)(R.r * kMaskWords + 1) * n + i] = m1;
            }
            if (staged) wave_sync();
        }
    }
    return over ? -1 : count;
}

// The neighbours of query i: from its masks when they exist and did not
// overflow, else by walking the cells.  visit4 hands each pair j's record
// to f(j, d, r2, code, q); visit reads separate component arrays and calls
// f(j, d, r2, code).
template <typename T, int D, typename S, typename F>
__device__ __forceinline__ void visit4(const Par<T>& P, const NbrMask& M, int64_t i,
                                       const int32_t* __restrict__ start, const S& src, const int c[3],
                                       const T oi[3], F&& f) {
    if (M.mask && M.count[i] >= 0) {
        mask_src<T, D>(P, start, src, c, oi, M.mask, M.n, i, f);
        return;
    }
    walk_src<T, D>(P, start, src, c, oi, f);
}

// The wall neighbours of fluid query i from its masks, for the pair sweeps:
// the same rows and ascending order as mask_src (so the same sums), with
// the wall's position record (wk) and, when nk is given, its normal record
// loaded one pair ahead, so each pair's gathers are in flight while the
// pair before it is computed.  f(w, d, r2, q, n) gets both records (n = 0
// without nk).  Queries whose masks overflowed walk the cells.
template <typename T, int D, typename F>
__device__ __forceinline__ void visit_walls(const Par<T>& P, const NbrMask& M, int64_t i,
                                            const int32_t* __restrict__ start, const Rec<T>* __restrict__ wk,
                                            const Rec<T>* __restrict__ nk, const int c[3], const T oi[3], F&& f) {
    auto nrm = [&](int j) { return nk ? ld4(nk, j) : Rec<T>{T(0), T(0), T(0), T(0)}; };
    if (!M.mask || M.count[i] < 0) {
        walk_src<T, D>(P, start, PackSrc<T>{wk}, c, oi,
                       [&](int j, const T* d, T r2, uint32_t, const Rec<T>& q) { f(j, d, r2, q, nrm(j)); });
        return;
    }
    for_rows<T, D>(P, start, c, oi, [&](const Row& R, T sy, T sz) {
        // cur: the bits still to visit of the current word (candidates
        // wb + bit), later: the row's second word
        uint64_t cur = M.mask[(int64_t)(R.r * kMaskWords + 0) * M.n + i];
        uint64_t later = R.j1 - R.base > 64 ? M.mask[(int64_t)(R.r * kMaskWords + 1) * M.n + i] : 0ull;
        int wb = R.base;
        if (cur == 0) {
            cur = later;
            later = 0;
            wb += 64;
        }
        if (cur == 0) return;
        int j = wb + __builtin_ctzll(cur);
        cur &= cur - 1;
        Rec<T> q = ld4(wk, j), n = nrm(j);
        while (true) {
            if (cur == 0 && later != 0) {
                cur = later;
                later = 0;
                wb += 64;
            }
            const bool more = cur != 0;
            const int jn = more ? wb + __builtin_ctzll(cur) : j;
            cur &= cur - 1;
            const Rec<T> qn = ld4(wk, jn), nn = nrm(jn);  // the next pair's records (this one's when last)
            T d[3];
            const T r2 = rel2<T, D>(oi, q.x, q.y, q.z, row_shift(j, R.jm, R.jp, P.L), sy, sz, d);
            f(j, d, r2, q, n);
            if (!more) break;
            j = jn;
            q = qn;
            n = nn;
        }
    });
}

template <typename T, int D, typename F>
__device__ __forceinline__ void visit(const Par<T>& P, const NbrMask& M, int64_t i,
                                      const int32_t* __restrict__ start, const T* __restrict__ o0,
                                      const T* __restrict__ o1, const T* __restrict__ o2,
                                      const int c[3], const T oi[3], F&& f) {
    visit4<T, D>(P, M, i, start, SoaSrc<T, D>{o0, o1, o2}, c, oi,
                 [&](int j, const T* d, T r2, uint32_t code, const Rec<T>&) { f(j, d, r2, code); });
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

// Distance of a pair in the neighbour sums: r^2 times its reciprocal square
// root, with the reciprocal root of 1 at r = 0 so that the self pair gives
// r = 0 exactly (one reciprocal root, no square root).  Every sum of W over
// neighbours takes this form, so the number density a sweep hands over is
// bit for bit the one the density update would sum.
template <typename T>
__device__ __forceinline__ T pair_r(T r2, T& rinv) {
    rinv = rsq(r2 > T(0) ? r2 : T(1));
    return r2 * rinv;
}

template <typename T>
__device__ __forceinline__ T pair_r(T r2) {
    T rinv;
    return pair_r(r2, rinv);
}

// W(r) and W'(r)/r from one t = 1 - q/2 (W exactly as wendland_W gives it).
template <typename T>
struct KernelWF {
    T W, F;
};

template <typename T>
__device__ __forceinline__ KernelWF<T> wendland_WF(const Par<T>& P, T r) {
    const T q = r * P.hinv;
    const T t = T(1) - T(0.5) * q;
    const T t2 = t * t;
    return KernelWF<T>{P.alpha * (t2 * t2) * (T(1) + T(2) * q), P.gfac * (t2 * t)};
}

}  // namespace sph
