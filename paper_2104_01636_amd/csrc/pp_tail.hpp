// pp_tail.hpp -- the small coarse levels of a multigrid cycle in one launch.
//
// Below a few thousand cells a grid launch per smoothing pass costs more than
// the pass itself, so the V-cycle over the last levels runs in one work-group
// of 1024 threads.  The iterates of every level and the whole operator of the
// levels after the first stay in LDS.  When the first level fits beside them
// its operator and right-hand side are staged in LDS as well, so the cycle
// waits for global memory once; otherwise (a first level of up to 8192 cells)
// they are read from global memory, where they are L2-resident.
// Each thread owns fixed x-pairs (2m, 2m+1) of the first level, with their
// indices and boundary flags computed once; a half-sweep touches only the cell
// of the pair that has the colour being relaxed.  Boundaries are handled
// without branches: a missing neighbour is replaced by the cell itself with a
// zero face weight.
//
// The arithmetic is that of the per-level kernels: red-black SOR from a zero
// guess (red, then black), pre/post sweeps, residual restricted by summing the
// 8 children, injection prolongation of the correction scaled by wc, and the
// dense inverse (or symmetric sweeps) on the last level.
#pragma once
#include <type_traits>

#include "pp_kernels.hpp"

namespace pp {

constexpr int kTailMaxLev = 12;
constexpr int kTailThreads = 1024;
constexpr int kTailMaxCells = 8192;                               // first tail level at most this large
constexpr int kTailSmallCells = 1200;                             // cells of the later levels (8192/7 < 1200)
constexpr int kTailDenseMax = 128;                                // rows of the dense inverse on the last level
constexpr int kTailDenseSplit = kTailThreads / kTailDenseMax;     // column chunks of its product

template <class T>
struct TailLevel {
    LevelView<T> v;  // operator in global memory
    T* rhs;          // right-hand side (first level: written by the restriction above)
    T* c;            // result (first level only)
    int n;
    int off;         // offset of a later level in the LDS arrays
};

template <class T>
struct TailDesc {
    int nlev;
    TailLevel<T> L[kTailMaxLev];
    const T* Minv;  // dense inverse of the last level (nd > 0), else symmetric sweeps
    int nd;
    T wc, omega;
    int nu, coarse_sweeps;
    int lds0;       // the first level's operator and right-hand side are staged in LDS
    int off0;       // their offset in the LDS arrays (after the later levels)
};

// x / d for 0 <= x < 2^22 and d > 0 from a float reciprocal, corrected to the
// exact quotient (the estimate is off by at most one).
__device__ inline int qdiv(int x, int d, float inv)
{
    int q = (int)((float)x * inv);
    const int r = x - q * d;
    q += (r >= d) - (r < 0);
    return q;
}

// Global load with a 32-bit byte offset (the tail's arrays are small).
template <class T>
__device__ inline T ldg(const T* base, int idx)
{
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + (unsigned)idx * (unsigned)sizeof(T));
}

// Neighbour flags of a cell: which in-plane neighbours exist, and whether the
// z neighbours wrap around the periodic seam.
enum : int { NB_W = 1, NB_E = 2, NB_S = 4, NB_N = 8, NB_ZLO = 16, NB_ZHI = 32 };

__device__ inline int nb_flags(int i, int j, int k, int nx, int ny, int nz)
{
    return (i > 0 ? NB_W : 0) | (i < nx - 1 ? NB_E : 0) | (j > 0 ? NB_S : 0) | (j < ny - 1 ? NB_N : 0) |
           (k == 0 ? NB_ZLO : 0) | (k == nz - 1 ? NB_ZHI : 0);
}

// Stencil sums s = sum W_f x_nb, d = sum W_f at cell c.  A supplies wx, wy, wz
// and x by index; every index used is inside the level.
template <class T, class A>
__device__ inline void tail_stencil(const A& a, int c, int fl, T& s, T& d)
{
    const int sy = a.nx, sz = a.nx * a.ny, wrap = (a.nz - 1) * sz;
    const int cw = (fl & NB_W) ? c - 1 : c, ce = (fl & NB_E) ? c + 1 : c;
    const int cs = (fl & NB_S) ? c - sy : c, cn = (fl & NB_N) ? c + sy : c;
    const int cb = (fl & NB_ZLO) ? c + wrap : c - sz, ct = (fl & NB_ZHI) ? c - wrap : c + sz;
    const T wwl = a.wx(cw), wsl = a.wy(cs);  // read unconditionally, then masked
    const T ww = (fl & NB_W) ? wwl : T(0), ws = (fl & NB_S) ? wsl : T(0);
    const T we = a.wx(c), wn = a.wy(c), wb = a.wz(cb), wt = a.wz(c);  // zero on wall faces
    s = ww * a.x(cw) + we * a.x(ce) + ws * a.x(cs) + wn * a.x(cn) + wb * a.x(cb) + wt * a.x(ct);
    d = ww + we + ws + wn + wb + wt;
}

// The first tail level: operator and right-hand side in global memory, x in LDS.
template <class T>
struct TailG {
    const T *gx, *gy, *gz, *gi, *gf;
    T* xs;
    int nx, ny, nz;
    __device__ T wx(int c) const { return ldg(gx, c); }
    __device__ T wy(int c) const { return ldg(gy, c); }
    __device__ T wz(int c) const { return ldg(gz, c); }
    __device__ T invd(int c) const { return ldg(gi, c); }
    __device__ T f(int c) const { return ldg(gf, c); }
    __device__ T x(int c) const { return xs[c]; }
};

// A later tail level: everything in LDS.
template <class T>
struct TailS {
    T *sx, *sy, *sz, *si, *sf, *xs;
    int nx, ny, nz;
    __device__ T wx(int c) const { return sx[c]; }
    __device__ T wy(int c) const { return sy[c]; }
    __device__ T wz(int c) const { return sz[c]; }
    __device__ T invd(int c) const { return si[c]; }
    __device__ T f(int c) const { return sf[c]; }
    __device__ T x(int c) const { return xs[c]; }
};

// Everything one relaxation of cell c reads, gathered before any of it is used.
template <class T>
struct TailIn {
    T ww, we, ws, wn, wb, wt;  // face weights (zero where there is no neighbour)
    T xw, xe, xs, xn, xb, xt;  // neighbour values
    T f, invd, xc;
};

template <class T, class A>
__device__ inline TailIn<T> tail_gather(const A& a, int c, int fl)
{
    const int sy = a.nx, sz = a.nx * a.ny, wrap = (a.nz - 1) * sz;
    const int cw = (fl & NB_W) ? c - 1 : c, ce = (fl & NB_E) ? c + 1 : c;
    const int cs = (fl & NB_S) ? c - sy : c, cn = (fl & NB_N) ? c + sy : c;
    const int cb = (fl & NB_ZLO) ? c + wrap : c - sz, ct = (fl & NB_ZHI) ? c - wrap : c + sz;
    TailIn<T> v;
    v.ww = a.wx(cw);
    v.ws = a.wy(cs);
    v.we = a.wx(c);
    v.wn = a.wy(c);
    v.wb = a.wz(cb);
    v.wt = a.wz(c);
    v.f = a.f(c);
    v.invd = a.invd(c);
    v.xw = a.x(cw);
    v.xe = a.x(ce);
    v.xs = a.x(cs);
    v.xn = a.x(cn);
    v.xb = a.x(cb);
    v.xt = a.x(ct);
    v.xc = a.x(c);
    if (!(fl & NB_W)) v.ww = T(0);
    if (!(fl & NB_S)) v.ws = T(0);
    return v;
}

template <class T>
__device__ inline T tail_update(const TailIn<T>& v, T omega)
{
    const T s = v.ww * v.xw + v.we * v.xe + v.ws * v.xs + v.wn * v.xn + v.wb * v.xb + v.wt * v.xt;
    T xv = (s + v.f) * v.invd;
    if (omega != T(1)) xv = v.xc + omega * (xv - v.xc);
    return xv;
}

template <class T, class A>
__device__ inline void tail_relax(const A& a, int c, int fl, T omega)
{
    T s, d;
    tail_stencil<T>(a, c, fl, s, d);
    T xv = (s + a.f(c)) * a.invd(c);
    if (omega != T(1)) xv = a.xs[c] + omega * (xv - a.xs[c]);
    a.xs[c] = xv;
}

// x-pairs of the first level, one packed int each in LDS: bits 0-12 the flat
// index of the even cell, bits 13-18 its neighbour flags, bit 19 (j + k) odd,
// bit 20 last pair of its row, bits 21-30 the coarse parent.
constexpr int kPairBits = 13;
static_assert(kTailMaxCells <= (1 << kPairBits) && kTailMaxCells / 8 <= (1 << 10), "pair packing");

template <class T>
__device__ inline void tail_pairs(const LevelView<T>& L, int* pinfo)
{
    const int hx = L.nx >> 1;
    const int np = hx * L.ny * L.nz;
    const float inv_hx = 1.0f / (float)hx, inv_ny = 1.0f / (float)L.ny;
    for (int t = threadIdx.x; t < np; t += kTailThreads) {
        const int row = qdiv(t, hx, inv_hx);
        const int m = t - row * hx;
        const int k = qdiv(row, L.ny, inv_ny);
        const int j = row - k * L.ny;
        const int fl = nb_flags(2 * m, j, k, L.nx, L.ny, L.nz) | (((j + k) & 1) << 6) | (m == hx - 1 ? 128 : 0);
        pinfo[t] = cell(L.nx, L.ny, 2 * m, j, k) | (fl << kPairBits) | (cell(hx, L.ny >> 1, m, j >> 1, k >> 1) << 21);
    }
}

// Cell of a packed pair with the given colour, and its neighbour flags.
__device__ inline void pair_cell(int pk, int colour, int& c, int& fl)
{
    const int f0 = (pk >> kPairBits) & 255;
    const int odd = ((f0 >> 6) ^ colour) & 1;  // 1: the odd cell of the pair has this colour
    c = (pk & ((1 << kPairBits) - 1)) + odd;
    // the even cell has a west neighbour iff m > 0 and always an east one; the
    // odd cell always a west one and an east one unless it ends the row
    fl = odd ? ((f0 & ~(NB_W | NB_E)) | NB_W | ((f0 & 128) ? 0 : NB_E)) : ((f0 & ~NB_E) | NB_E);
}

// Half-sweep of the first level: NB pairs per thread and round, all loads of
// their cells issued before any is computed (the cells of one colour are
// independent).
template <int NB, class T, class A>
__device__ inline void tail_half_first_n(const A& a, const int* pinfo, int np, int colour, T omega)
{
    for (int t = threadIdx.x; t < np; t += NB * kTailThreads) {
        int c[NB], fl[NB];
        TailIn<T> v[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int tb = t + b * kTailThreads;
            pair_cell(pinfo[tb < np ? tb : t], colour, c[b], fl[b]);
            v[b] = tail_gather<T>(a, c[b], fl[b]);
        }
        __builtin_amdgcn_sched_barrier(0);  // keep all loads ahead of the arithmetic
        T x[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) x[b] = tail_update(v[b], omega);
#pragma unroll
        for (int b = 0; b < NB; ++b)
            if (t + b * kTailThreads < np) a.xs[c[b]] = x[b];
    }
}

// The batch is the pairs per thread the level has, up to 4 in float32 and 2 in
// float64 (as registers allow): a batch slot beyond the last pair would gather
// again for nothing.
template <class T, class A>
__device__ inline void tail_half_first(const A& a, const int* pinfo, int np, int colour, T omega)
{
    if (np <= kTailThreads) tail_half_first_n<1, T>(a, pinfo, np, colour, omega);
    else if (sizeof(T) == 8 || np <= 2 * kTailThreads) tail_half_first_n<2, T>(a, pinfo, np, colour, omega);
    else tail_half_first_n<4, T>(a, pinfo, np, colour, omega);
    __syncthreads();
}

// Half-sweep of a later level (nx even: x-pairs, at most one per thread here).
template <class T>
__device__ inline void tail_half_small(const TailS<T>& a, int colour, T omega)
{
    const int hx = a.nx >> 1;
    const int np = hx * a.ny * a.nz;
    const float inv_hx = 1.0f / (float)hx, inv_ny = 1.0f / (float)a.ny;
    for (int t = threadIdx.x; t < np; t += kTailThreads) {
        const int row = qdiv(t, hx, inv_hx);
        const int m = t - row * hx;
        const int k = qdiv(row, a.ny, inv_ny);
        const int j = row - k * a.ny;
        const int i = 2 * m + ((j + k + colour) & 1);
        tail_relax<T>(a, cell(a.nx, a.ny, i, j, k), nb_flags(i, j, k, a.nx, a.ny, a.nz), omega);
    }
    __syncthreads();
}

// The same for any nx (the last level when it is smoothed instead of solved).
template <class T>
__device__ inline void tail_half_any(const TailS<T>& a, int n, int colour, T omega)
{
    const float inv_nx = 1.0f / (float)a.nx, inv_ny = 1.0f / (float)a.ny;
    for (int c = threadIdx.x; c < n; c += kTailThreads) {
        const int row = qdiv(c, a.nx, inv_nx);
        const int i = c - row * a.nx;
        const int k = qdiv(row, a.ny, inv_ny);
        const int j = row - k * a.ny;
        if (((i + j + k) & 1) != colour) continue;
        tail_relax<T>(a, c, nb_flags(i, j, k, a.nx, a.ny, a.nz), omega);
    }
    __syncthreads();
}

// Residual of level a summed over the 8 children of coarse cell (I, J, K).
template <class T, class A>
__device__ inline T tail_restrict_cell(const A& a, int I, int J, int K)
{
    T acc = T(0);
#pragma unroll 1
    for (int dk = 0; dk < 2; ++dk)
        for (int dj = 0; dj < 2; ++dj)
            for (int di = 0; di < 2; ++di) {
                const int i = 2 * I + di, j = 2 * J + dj, k = 2 * K + dk;
                const int c = cell(a.nx, a.ny, i, j, k);
                T s, d;
                tail_stencil<T>(a, c, nb_flags(i, j, k, a.nx, a.ny, a.nz), s, d);
                acc += a.f(c) - (d * a.x(c) - s);
            }
    return acc;
}

template <class T, class A>
__device__ inline void tail_restrict(const A& a, T* fc, int cnx, int cny, int cn)
{
    const float inv_cx = 1.0f / (float)cnx, inv_cy = 1.0f / (float)cny;
    for (int cc = threadIdx.x; cc < cn; cc += kTailThreads) {
        const int row = qdiv(cc, cnx, inv_cx);
        const int I = cc - row * cnx;
        const int K = qdiv(row, cny, inv_cy);
        const int J = row - K * cny;
        fc[cc] = tail_restrict_cell<T>(a, I, J, K);
    }
    __syncthreads();
}

// The same for a level of at most kTailThreads cells: every thread forms one
// cell's residual into rbuf, then each coarse cell adds its 8 children in the
// order tail_restrict_cell does (the same sums, without its serial chain).
template <class T, class A>
__device__ inline void tail_restrict_wide(const A& a, T* rbuf, T* fc, int cnx, int cny, int cn)
{
    const int n = a.nx * a.ny * a.nz;
    const float inv_nx = 1.0f / (float)a.nx, inv_ny = 1.0f / (float)a.ny;
    for (int c = threadIdx.x; c < n; c += kTailThreads) {
        const int row = qdiv(c, a.nx, inv_nx);
        const int i = c - row * a.nx;
        const int k = qdiv(row, a.ny, inv_ny);
        const int j = row - k * a.ny;
        T s, d;
        tail_stencil<T>(a, c, nb_flags(i, j, k, a.nx, a.ny, a.nz), s, d);
        rbuf[c] = a.f(c) - (d * a.x(c) - s);
    }
    __syncthreads();
    const float inv_cx = 1.0f / (float)cnx, inv_cy = 1.0f / (float)cny;
    for (int cc = threadIdx.x; cc < cn; cc += kTailThreads) {
        const int row = qdiv(cc, cnx, inv_cx);
        const int I = cc - row * cnx;
        const int K = qdiv(row, cny, inv_cy);
        const int J = row - K * cny;
        T acc = T(0);
#pragma unroll
        for (int dk = 0; dk < 2; ++dk)
#pragma unroll
            for (int dj = 0; dj < 2; ++dj)
#pragma unroll
                for (int di = 0; di < 2; ++di) acc += rbuf[cell(a.nx, a.ny, 2 * I + di, 2 * J + dj, 2 * K + dk)];
        fc[cc] = acc;
    }
    __syncthreads();
}

// x += wc * e(parent) on every cell of a later level (nx even).
template <class T>
__device__ inline void tail_prolong_small(const TailS<T>& a, const T* e, T wc)
{
    const int hx = a.nx >> 1;
    const int np = hx * a.ny * a.nz;
    const float inv_hx = 1.0f / (float)hx, inv_ny = 1.0f / (float)a.ny;
    for (int t = threadIdx.x; t < np; t += kTailThreads) {
        const int row = qdiv(t, hx, inv_hx);
        const int m = t - row * hx;
        const int k = qdiv(row, a.ny, inv_ny);
        const int j = row - k * a.ny;
        const int c0 = cell(a.nx, a.ny, 2 * m, j, k);
        const T ev = wc * e[cell(hx, a.ny >> 1, m, j >> 1, k >> 1)];
        a.xs[c0] += ev;
        a.xs[c0 + 1] += ev;
    }
    __syncthreads();
}

// One V-cycle over the levels of D from a zero guess at the top; the result is
// left in D.L[0].c.  LDS0: the first level's operator and right-hand side are
// staged in LDS (D.lds0) instead of read from global memory.
// (one block of 16 wavefronts: 4 per SIMD is all the occupancy there is, so the
// compiler may spend registers on keeping loads in flight)
template <class T, bool LDS0>
__global__ void __launch_bounds__(kTailThreads) __attribute__((amdgpu_waves_per_eu(1, 4))) k_tail_vcycle(TailDesc<T> D)
{
    __shared__ T x0[kTailMaxCells];
    __shared__ T sxs[kTailSmallCells], swx[kTailSmallCells], swy[kTailSmallCells], swz[kTailSmallCells],
        sid[kTailSmallCells], sf[kTailSmallCells];
    __shared__ int pinfo[kTailMaxCells / 2];
    __shared__ T dpart[kTailThreads];
    const int last = D.nlev - 1;
    const T om = D.omega;
    const TailLevel<T>& V0 = D.L[0];

    // the dense inverse's entries this thread multiplies on the last level (see
    // below), loaded now so that their latency overlaps the staging
    constexpr int kPer = kTailDenseMax / kTailDenseSplit;
    const int dr = threadIdx.x % kTailDenseMax, dc0 = (threadIdx.x / kTailDenseMax) * kPer;
    T m[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int c = dc0 + u;
        m[u] = (dr < D.nd && c < D.nd) ? ldg(D.Minv, c * D.nd + dr) : T(0);
    }

    // stage the operators of the later levels (and, with LDS0, the first level's
    // operator and right-hand side after them): every load of the cycle but the
    // dense inverse is issued here, all of them before the first is stored
    {
        static_assert(kTailSmallCells <= 2 * kTailThreads, "two staged cells per thread and group");
        T lw[2][4], fw[2][5];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int e = threadIdx.x + u * kTailThreads;  // index into the later levels' LDS arrays
            if (e < D.off0) {
                // level of e: the last later level whose range starts at or before e
                const T *px = nullptr, *py = nullptr, *pz = nullptr, *pi = nullptr;
                int base = 0;
#pragma unroll
                for (int l = 1; l < kTailMaxLev; ++l) {
                    if (l <= last && e >= D.L[l].off) {
                        px = D.L[l].v.wx;
                        py = D.L[l].v.wy;
                        pz = D.L[l].v.wz;
                        pi = D.L[l].v.invd;
                        base = D.L[l].off;
                    }
                }
                lw[u][0] = ldg(px, e - base);
                lw[u][1] = ldg(py, e - base);
                lw[u][2] = ldg(pz, e - base);
                lw[u][3] = ldg(pi, e - base);
            }
            if constexpr (LDS0) {
                if (e < V0.n) {
                    fw[u][0] = ldg(V0.v.wx, e);
                    fw[u][1] = ldg(V0.v.wy, e);
                    fw[u][2] = ldg(V0.v.wz, e);
                    fw[u][3] = ldg(V0.v.invd, e);
                    fw[u][4] = ldg(V0.rhs, e);
                }
            }
        }
        __builtin_amdgcn_sched_barrier(0);  // every load in flight before the first store waits
        tail_pairs(V0.v, pinfo);            // formed while the loads are in flight
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int e = threadIdx.x + u * kTailThreads;
            if (e < D.off0) {
                swx[e] = lw[u][0];
                swy[e] = lw[u][1];
                swz[e] = lw[u][2];
                sid[e] = lw[u][3];
            }
            if constexpr (LDS0) {
                if (e < V0.n) {
                    swx[D.off0 + e] = fw[u][0];
                    swy[D.off0 + e] = fw[u][1];
                    swz[D.off0 + e] = fw[u][2];
                    sid[D.off0 + e] = fw[u][3];
                    sf[D.off0 + e] = fw[u][4];
                }
            }
        }
    }
#define PP_TAIL_SMALL(l)                                                                                          \
    TailS<T>{swx + D.L[l].off, swy + D.L[l].off, swz + D.L[l].off, sid + D.L[l].off, sf + D.L[l].off, sxs + D.L[l].off, \
             D.L[l].v.nx, D.L[l].v.ny, D.L[l].v.nz}

    // first level: pairs, sweeps from zero, restriction into level 1
    using First = std::conditional_t<LDS0, TailS<T>, TailG<T>>;
    First g;
    if constexpr (LDS0) {
        g = TailS<T>{swx + D.off0, swy + D.off0, swz + D.off0, sid + D.off0, sf + D.off0, x0, V0.v.nx, V0.v.ny, V0.v.nz};
    } else {
        g = TailG<T>{V0.v.wx, V0.v.wy, V0.v.wz, V0.v.invd, V0.rhs, x0, V0.v.nx, V0.v.ny, V0.v.nz};
    }
    const int np0 = V0.n >> 1;
    __syncthreads();  // completes the staging and the pairs above
#pragma unroll 2
    for (int t = threadIdx.x; t < np0; t += kTailThreads) {
        int c, fl;
        pair_cell(pinfo[t], 0, c, fl);
        x0[c] = om * (g.f(c) * g.invd(c));
        x0[c ^ 1] = T(0);  // the even cell's index is even: the pair's cells differ in the lowest bit
    }
    __syncthreads();
    tail_half_first(g, pinfo, np0, 1, om);
    for (int s = 1; s < D.nu; ++s) {
        tail_half_first(g, pinfo, np0, 0, om);
        tail_half_first(g, pinfo, np0, 1, om);
    }
    if (V0.n <= kTailThreads) tail_restrict_wide<T>(g, dpart, sf + D.L[1].off, D.L[1].v.nx, D.L[1].v.ny, D.L[1].n);
    else tail_restrict<T>(g, sf + D.L[1].off, D.L[1].v.nx, D.L[1].v.ny, D.L[1].n);

    // later levels down to the last
    for (int l = 1; l < last; ++l) {
        const TailS<T> a = PP_TAIL_SMALL(l);
        const int np = (a.nx >> 1) * a.ny * a.nz;
        const float inv_hx = 1.0f / (float)(a.nx >> 1), inv_ny = 1.0f / (float)a.ny;
        for (int t = threadIdx.x; t < np; t += kTailThreads) {
            const int row = qdiv(t, a.nx >> 1, inv_hx);
            const int m = t - row * (a.nx >> 1);
            const int k = qdiv(row, a.ny, inv_ny);
            const int j = row - k * a.ny;
            const int c0 = cell(a.nx, a.ny, 2 * m, j, k);
            const int cr = c0 + ((j + k) & 1);
            a.xs[cr] = om * (a.f(cr) * a.invd(cr));
            a.xs[cr ^ 1] = T(0);
        }
        __syncthreads();
        tail_half_small(a, 1, om);
        for (int s = 1; s < D.nu; ++s) {
            tail_half_small(a, 0, om);
            tail_half_small(a, 1, om);
        }
        const TailS<T> cN = PP_TAIL_SMALL(l + 1);
        if (D.L[l].n <= kTailThreads) tail_restrict_wide<T>(a, dpart, cN.sf, cN.nx, cN.ny, D.L[l + 1].n);
        else tail_restrict<T>(a, cN.sf, cN.nx, cN.ny, D.L[l + 1].n);
    }
    {
        const TailS<T> b = PP_TAIL_SMALL(last);
        const int n = D.L[last].n;
        if (D.nd > 0) {
            // x = Minv f (nd <= kTailDenseMax): thread t forms row t mod kTailDenseMax
            // over one chunk of the columns, with all of its loads issued together;
            // the chunks are then added in a fixed order
            const int nd = D.nd;
            T acc = T(0);
#pragma unroll
            for (int u = 0; u < kPer; ++u) {
                const int c = dc0 + u;
                acc += m[u] * (c < nd ? b.sf[c] : T(0));
            }
            dpart[threadIdx.x] = acc;
            __syncthreads();
            if (threadIdx.x < nd) {
                T x = T(0);
#pragma unroll
                for (int h = 0; h < kTailDenseSplit; ++h) x += dpart[h * kTailDenseMax + threadIdx.x];
                b.xs[threadIdx.x] = x;
            }
            __syncthreads();
        } else {
            for (int c = threadIdx.x; c < n; c += kTailThreads) b.xs[c] = T(0);
            __syncthreads();
            for (int s = 0; s < D.coarse_sweeps; ++s) {
                tail_half_any(b, n, 0, om);
                tail_half_any(b, n, 1, om);
            }
            for (int s = 0; s < D.coarse_sweeps; ++s) {
                tail_half_any(b, n, 1, om);
                tail_half_any(b, n, 0, om);
            }
        }
    }
    // back up: prolongation and correction of every cell, then black before red
    for (int l = last - 1; l >= 1; --l) {
        const TailS<T> a = PP_TAIL_SMALL(l);
        tail_prolong_small(a, PP_TAIL_SMALL(l + 1).xs, D.wc);
        for (int s = 0; s < D.nu; ++s) {
            tail_half_small(a, 1, om);
            tail_half_small(a, 0, om);
        }
    }
    {
        const T* e = sxs + D.L[1].off;
#pragma unroll 2
        for (int t = threadIdx.x; t < np0; t += kTailThreads) {
            const int pk = pinfo[t];
            const int c0 = pk & ((1 << kPairBits) - 1);
            const T ev = D.wc * e[pk >> 21];
            x0[c0] += ev;
            x0[c0 + 1] += ev;
        }
        __syncthreads();
        for (int s = 0; s < D.nu; ++s) {
            tail_half_first(g, pinfo, np0, 1, om);
            tail_half_first(g, pinfo, np0, 0, om);
        }
    }
    for (int c = threadIdx.x; c < V0.n; c += kTailThreads) V0.c[c] = x0[c];
#undef PP_TAIL_SMALL
}

}  // namespace pp
