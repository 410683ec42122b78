// pp_kernels.hpp -- HIP kernels (gfx950) for the variable-density pressure solve.
//
// The pressure equation (Kumar & Vanka, arXiv 2104.01636, Section 2.2, step 11)
//     div( grad(p) / rho ) = div(u_f) / dt
// is discretised on a uniform cell-centred grid with face coefficients
// beta_f = 2/(rho_L + rho_R) (cell-to-face linear averaging of rho, the note
// after the step list), walls in x and y and periodicity in z (Section 4).
// Internally every level solves K x = f with the positive semi-definite
//     (K x)_c = D_c x_c - sum_f W_f x_nb(f),   D_c = sum_f W_f,
// where on the finest level W_f = beta_f (so K = -h^2 A) and on coarse levels
// W_f is the sum of the four fine faces that form the coarse face (the
// Galerkin product P^T K P for injection prolongation P).  Face weights are
// computed once per density and stored: W_x[c] is the +x face of cell c (zero
// on the wall face i = nx-1), W_y likewise, W_z[c] the +z face (the last plane's
// face joins plane 0).  The solve kernels therefore do no divisions.
//
// Layout: flat index i + nx*(j + ny*k), x fastest; 32-bit indices (a level has
// fewer than 2^31 cells).  Grid kernels run a 2-D tile of threads over (x, y)
// and march a contiguous range of z planes per block, so the z neighbours of a
// plane were touched by the same block one step before.
//
// Reductions accumulate in float64 whatever the vector precision: each block
// reduces with wavefront shuffles and LDS, writes its partial, and the last
// block to finish sums all partials in a fixed order.  Results therefore do
// not depend on scheduling (bitwise repeatable).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace pp {

constexpr int kBlock = 256;          // threads per block for grid kernels
constexpr int kMaxRedBlocks = 2048;  // blocks of a reducing launch, at most (the per-plane launches)
constexpr int kMaxPartialBlocks = 4096;  // ... and of any reducing launch (the size of the partials buffer)
constexpr int kMaxRed = 4;           // values reduced by one launch

// Operator of one level, in precision T.
template <class T>
struct LevelView {
    int nx, ny, nz;
    const T* wx;    // +x face weight of each cell (0 on the wall face)
    const T* wy;
    const T* wz;    // +z face weight (the last plane's face joins plane 0)
    const T* invd;  // 1 / D_c
    const T* rho = nullptr;  // finest level: density, from which the plane-marching kernels derive the weights
    // bfloat16 copies of wx, wy, wz that the plane-marching kernels read instead
    // (coarse levels of the float32 preconditioner), or null
    const unsigned short* hwx = nullptr;
    const unsigned short* hwy = nullptr;
    const unsigned short* hwz = nullptr;
};

// bfloat16: the upper 16 bits of an IEEE binary32 value, here rounded to
// nearest (ties to even) from the lower 16; the float32 exponent range with 8
// significant bits.  Only finite values are converted.
__device__ inline unsigned short to_bf16(float x)
{
    unsigned u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ inline float from_bf16(unsigned short b) { return __uint_as_float((unsigned)b << 16); }

// Reduction target: per-block partials and the output slots.  A reducing
// launch writes one partial per block; k_reduce_finish, launched after it on
// the same stream, sums them in a fixed order.
struct Reduce {
    double* partials;    // [kMaxPartialBlocks * kMaxRed]
    double* out;         // scalar slots receiving the totals
    int slot[kMaxRed];   // slot index per reduced value
    double* host = nullptr;  // device view of mapped pinned host slots that also receive the totals
                             // (totals the host reads: no copy launch after the reduction), or null
};

// Scalars a kernel reads from the device slot array (no host round trip).
struct Coefs {
    const double* s;   // slot array
    int num, den;      // factor = sign * s[num] / s[den]   (den < 0: factor = sign * s[num])
    double sign;
    int c1 = -1, c2 = -1;  // with c1 >= 0 the numerator is s[num] + cs * s[c1] * s[c2]
    double cs = 0.0;
    __device__ inline double get() const
    {
        const double nv = c1 >= 0 ? s[num] + cs * s[c1] * s[c2] : s[num];
        return den < 0 ? sign * nv : sign * nv / s[den];
    }
};

__device__ inline int cell(int nx, int ny, int i, int j, int k) { return i + nx * (j + ny * k); }

// s = sum_f W_f val(nb(f)), d = sum_f W_f; val(m, i, j, k) gets the neighbour's
// flat index and coordinates.
template <class T, class F>
__device__ inline void nbsum(const LevelView<T>& L, int i, int j, int k, int c, F val, T& s, T& d)
{
    const int sy = L.nx, sz = L.nx * L.ny;
    const int kb = k > 0 ? k - 1 : L.nz - 1, kt = k < L.nz - 1 ? k + 1 : 0;
    const int cb = c + (kb - k) * sz, ct = c + (kt - k) * sz;
    T ss = T(0), dd = T(0);
    if (i > 0) { T w = L.wx[c - 1]; ss += w * val(c - 1, i - 1, j, k); dd += w; }
    if (i < L.nx - 1) { T w = L.wx[c]; ss += w * val(c + 1, i + 1, j, k); dd += w; }
    if (j > 0) { T w = L.wy[c - sy]; ss += w * val(c - sy, i, j - 1, k); dd += w; }
    if (j < L.ny - 1) { T w = L.wy[c]; ss += w * val(c + sy, i, j + 1, k); dd += w; }
    { T w = L.wz[cb]; ss += w * val(cb, i, j, kb); dd += w; }
    { T w = L.wz[c]; ss += w * val(ct, i, j, kt); dd += w; }
    s = ss;
    d = dd;
}

// ---------------------------------------------------------------- reductions

__device__ inline double wave_sum(double x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// Block-reduce NV values and store the block's partials.  Every thread of the
// block must call this.  There is no grid-wide completion step in the kernel:
// an agent-scope fence per block would write back and invalidate the L2 of
// its XCD, so the totals are formed by k_reduce_finish after the launch.
template <int NV>
__device__ inline void reduce_finish(double (&v)[NV], const Reduce& R)
{
    __shared__ double sh[NV][16];  // up to 1024 threads
    const int nthr = blockDim.x * blockDim.y * blockDim.z;
    const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    const int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    const int nw = (nthr + 63) / 64;
#pragma unroll
    for (int m = 0; m < NV; ++m) {
        double x = wave_sum(v[m]);
        if ((tid & 63) == 0) sh[m][tid >> 6] = x;
    }
    __syncthreads();
    if (tid == 0) {
#pragma unroll
        for (int m = 0; m < NV; ++m) {
            double t = 0.0;
            for (int w = 0; w < nw; ++w) t += sh[m][w];
            R.partials[(size_t)bid * kMaxRed + m] = t;
        }
    }
}

// Totals of a reducing launch of nblk blocks: partials summed thread-strided,
// then by wavefront and across wavefronts, always in the same order.  One block.
__global__ void __launch_bounds__(kBlock) k_reduce_finish(Reduce R, int nblk, int nv)
{
    __shared__ double sh[kBlock / 64];
    for (int m = 0; m < nv; ++m) {
        double t = 0.0;
        for (int b = threadIdx.x; b < nblk; b += kBlock) t += R.partials[(size_t)b * kMaxRed + m];
        t = wave_sum(t);
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = t;
        __syncthreads();
        if (threadIdx.x == 0) {
            double tot = 0.0;
            for (int w = 0; w < kBlock / 64; ++w) tot += sh[w];
            R.out[R.slot[m]] = tot;
            if (R.host) R.host[R.slot[m]] = tot;
        }
        __syncthreads();
    }
}

// Tile geometry: threads (x, y) in the block, block z covers planes [k0, k1).
struct Tile {
    int i, j, k0, k1;
    bool act;
};
__device__ inline Tile tile(int nx, int ny, int nz, int kper)
{
    Tile t;
    t.i = blockIdx.x * blockDim.x + threadIdx.x;
    t.j = blockIdx.y * blockDim.y + threadIdx.y;
    t.k0 = blockIdx.z * kper;
    t.k1 = min(nz, t.k0 + kper);
    t.act = t.i < nx && t.j < ny;
    return t;
}

// ---------------------------------------------------------------- smoothing

// Red-black SOR from a zero guess: red cells (i+j+k even) get omega f/D, black
// cells one update from their red neighbours (computed on the fly).
template <class T>
__global__ void __launch_bounds__(kBlock) k_smooth_first(LevelView<T> L, const T* __restrict__ f, T* __restrict__ x, int kper,
                                                        T omega)
{
    Tile t = tile(L.nx, L.ny, L.nz, kper);
    if (!t.act) return;
    for (int k = t.k0; k < t.k1; ++k) {
        const int c = cell(L.nx, L.ny, t.i, t.j, k);
        if (((t.i + t.j + k) & 1) == 0) {
            x[c] = omega * (f[c] * L.invd[c]);
        } else {
            T s, d;
            nbsum<T>(L, t.i, t.j, k, c, [&](int m, int, int, int) { return omega * (f[m] * L.invd[m]); }, s, d);
            x[c] = omega * ((s + f[c]) * L.invd[c]);
        }
    }
}

// One SOR half-sweep over one colour, in place.  With NDOT > 0 the launch also
// reduces sum(x) (and <x, q> for NDOT >= 2, <x, f> for NDOT >= 3, sum(f) for
// NDOT = 4) over all cells after the update.
template <class T, int NDOT, class TQ = T>
__global__ void __launch_bounds__(kBlock) k_smooth_half(LevelView<T> L, const T* __restrict__ f, T* x, int colour, int kper,
                                                       const TQ* __restrict__ q, Reduce R, T omega)
{
    Tile t = tile(L.nx, L.ny, L.nz, kper);
    double acc[NDOT > 0 ? NDOT : 1] = {};
    if (t.act) {
        for (int k = t.k0; k < t.k1; ++k) {
            const int c = cell(L.nx, L.ny, t.i, t.j, k);
            T xv;
            if (((t.i + t.j + k) & 1) == colour) {
                T s, d;
                nbsum<T>(L, t.i, t.j, k, c, [&](int m, int, int, int) { return x[m]; }, s, d);
                xv = (s + f[c]) * L.invd[c];
                if (omega != T(1)) xv = x[c] + omega * (xv - x[c]);
                x[c] = xv;
            } else {
                xv = x[c];
            }
            if constexpr (NDOT >= 1) acc[0] += (double)xv;
            if constexpr (NDOT >= 2) acc[1] += (double)xv * (double)q[c];
            if constexpr (NDOT >= 3) acc[2] += (double)xv * (double)f[c];
            if constexpr (NDOT >= 4) acc[3] += (double)f[c];
        }
    }
    if constexpr (NDOT > 0) reduce_finish<NDOT>(acc, R);
}

// Restriction of the residual: rhs_c(I,J,K) = sum over the 8 children of (f - K x).
template <class T>
__global__ void __launch_bounds__(kBlock) k_residual_restrict(LevelView<T> L, const T* __restrict__ f, const T* __restrict__ x,
                                                             T* __restrict__ rc, int cnx, int cny, int cnz, int kper)
{
    Tile t = tile(cnx, cny, cnz, kper);
    if (!t.act) return;
    for (int K = t.k0; K < t.k1; ++K) {
        T acc = T(0);
#pragma unroll 1
        for (int dk = 0; dk < 2; ++dk)
#pragma unroll
            for (int dj = 0; dj < 2; ++dj)
#pragma unroll
                for (int di = 0; di < 2; ++di) {
                    const int i = 2 * t.i + di, j = 2 * t.j + dj, k = 2 * K + dk;
                    const int c = cell(L.nx, L.ny, i, j, k);
                    T s, d;
                    nbsum<T>(L, i, j, k, c, [&](int m, int, int, int) { return x[m]; }, s, d);
                    acc += f[c] - (d * x[c] - s);
                }
        rc[cell(cnx, cny, t.i, t.j, K)] = acc;
    }
}

// Out of place: y = x + wc * P e on red cells, then one black SOR half-sweep
// that sees the corrected red values.
template <class T>
__global__ void __launch_bounds__(kBlock) k_prolong_black(LevelView<T> L, const T* __restrict__ f, const T* __restrict__ x,
                                                         const T* __restrict__ e, T wc, T* __restrict__ y, int kper, T omega)
{
    Tile t = tile(L.nx, L.ny, L.nz, kper);
    if (!t.act) return;
    const int cnx = L.nx >> 1, cny = L.ny >> 1;
    auto xe = [&](int m, int i, int j, int k) { return x[m] + wc * e[cell(cnx, cny, i >> 1, j >> 1, k >> 1)]; };
    for (int k = t.k0; k < t.k1; ++k) {
        const int c = cell(L.nx, L.ny, t.i, t.j, k);
        const T xo = x[c] + wc * e[cell(cnx, cny, t.i >> 1, t.j >> 1, k >> 1)];
        if (((t.i + t.j + k) & 1) == 0) {
            y[c] = xo;
        } else {
            T s, d;
            nbsum<T>(L, t.i, t.j, k, c, xe, s, d);
            T gs = (s + f[c]) * L.invd[c];
            if (omega != T(1)) gs = xo + omega * (gs - xo);
            y[c] = gs;
        }
    }
}

// ---------------------------------------------------------------- Krylov steps

// d_new = (z - m) + b * d_old, q = K d_new; reduces <d_new, q> and <d_new, r>
// (FINE: <d_new, q> only).
// m = s[msum]/n (mean projection, finest level only) and b from the slots.  The
// preconditioned residual z may be stored in a lower precision TZ than d and q.
// FINE (the finest level's Krylov step): also applies the previous step's
// deferred x += ap * d_old (when use_beta, i.e. after the first step).
template <class T, class TZ = T, bool FINE = false>
__global__ void __launch_bounds__(kBlock) k_dir_apply(LevelView<T> L, const TZ* __restrict__ z, const T* __restrict__ dold,
                                                     T* __restrict__ dnew, T* __restrict__ q, const T* __restrict__ r,
                                                     T* __restrict__ x, Coefs beta, int use_beta, Coefs mean, int use_mean,
                                                     Coefs aprev, int kper, Reduce R)
{
    Tile t = tile(L.nx, L.ny, L.nz, kper);
    const T b = use_beta ? (T)beta.get() : T(0);
    const T m = use_mean ? (T)mean.get() : T(0);
    const T ap = (FINE && use_beta) ? (T)aprev.get() : T(0);
    double acc[FINE ? 1 : 2] = {};
    if (t.act) {
        auto dv = [&](int c, int, int, int) { return use_beta ? ((T)z[c] - m) + b * dold[c] : ((T)z[c] - m); };
        for (int k = t.k0; k < t.k1; ++k) {
            const int c = cell(L.nx, L.ny, t.i, t.j, k);
            T s, d;
            nbsum<T>(L, t.i, t.j, k, c, dv, s, d);
            const T dc = dv(c, 0, 0, 0);
            const T qc = d * dc - s;
            dnew[c] = dc;
            q[c] = qc;
            acc[0] += (double)dc * (double)qc;
            if constexpr (!FINE) acc[1] += (double)dc * (double)r[c];
            if constexpr (FINE) {
                if (use_beta) x[c] = x[c] + ap * dold[c];
            }
        }
    }
    reduce_finish<FINE ? 1 : 2>(acc, R);
}

// x += a d (or x = a d when first; only with do_x), r -= a q (unless skip_r);
// reduces ||r||^2 and sum(r); with r32 also writes the float32 copy of r.  n is even (every level
// has an even number of planes): a thread handles pairs of cells with 2-wide
// loads, two pairs per trip.
template <class T> struct Vec2;
template <> struct Vec2<float> { using type = float2; };
template <> struct Vec2<double> { using type = double2; };

template <class T>
__global__ void __launch_bounds__(kBlock) k_update_xr(int n, T* __restrict__ x, const T* __restrict__ d, T* __restrict__ r,
                                                     const T* __restrict__ q, Coefs alpha, int first, int skip_r, int want_red,
                                                     Reduce R, float* __restrict__ r32, int do_x,
                                                     double* __restrict__ alpha_out = nullptr)
{
    using V = typename Vec2<T>::type;
    const double ad = alpha.get();
    const T a = (T)ad;
    if (alpha_out && blockIdx.x == 0 && threadIdx.x == 0) *alpha_out = ad;  // for the deferred x update
    double acc[2] = {0.0, 0.0};
    const int np = n >> 1;
    const int stride = gridDim.x * blockDim.x;
    V* x2 = reinterpret_cast<V*>(x);
    const V* d2 = reinterpret_cast<const V*>(d);
    V* r2 = reinterpret_cast<V*>(r);
    const V* q2 = reinterpret_cast<const V*>(q);
    float2* s2 = reinterpret_cast<float2*>(r32);
#pragma unroll 2
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < np; p += stride) {
        if (do_x) {
            const V dv = d2[p];
            V xv;
            if (first) {
                xv.x = a * dv.x;
                xv.y = a * dv.y;
            } else {
                xv = x2[p];
                xv.x = xv.x + a * dv.x;
                xv.y = xv.y + a * dv.y;
            }
            x2[p] = xv;
        }
        if (!skip_r) {
            V rv = r2[p];
            const V qv = q2[p];
            rv.x = rv.x - a * qv.x;
            rv.y = rv.y - a * qv.y;
            r2[p] = rv;
            if (r32) s2[p] = make_float2((float)rv.x, (float)rv.y);
            acc[0] += (double)rv.x * (double)rv.x;
            acc[0] += (double)rv.y * (double)rv.y;
            acc[1] += (double)rv.x;
            acc[1] += (double)rv.y;
        }
    }
    if (want_red) reduce_finish<2>(acc, R);
}

// r = f - K x on any level from its stored face weights (one thread per cell
// column): the coarse residual of a W-cycle's second visit.
template <class T>
__global__ void __launch_bounds__(kBlock) k_residual(LevelView<T> L, const T* __restrict__ f, const T* __restrict__ x,
                                                    T* __restrict__ r, int kper)
{
    const Tile t = tile(L.nx, L.ny, L.nz, kper);
    if (!t.act) return;
    for (int k = t.k0; k < t.k1; ++k) {
        const int c = cell(L.nx, L.ny, t.i, t.j, k);
        T s, d;
        nbsum<T>(L, t.i, t.j, k, c, [&](int m, int, int, int) { return x[m]; }, s, d);
        r[c] = f[c] - (d * x[c] - s);
    }
}

// Coarsest level: x = M f with the dense symmetric matrix M (one block).
template <class T>
__global__ void __launch_bounds__(kBlock) k_dense_apply(int n, const T* __restrict__ M, const T* __restrict__ f, T* __restrict__ x)
{
    __shared__ T fs[kBlock];
    for (int r0 = 0; r0 < n; r0 += kBlock) {
        const int r = r0 + threadIdx.x;
        T acc = T(0);
        for (int c0 = 0; c0 < n; c0 += kBlock) {
            __syncthreads();
            if (c0 + threadIdx.x < n) fs[threadIdx.x] = f[c0 + threadIdx.x];
            __syncthreads();
            const int cm = min(kBlock, n - c0);
            if (r < n)
                for (int c = 0; c < cm; ++c) acc += M[(c0 + c) * n + r] * fs[c];
        }
        if (r < n) x[r] = acc;
    }
}


// ---------------------------------------------------------------- float64 outer pieces

// r = f - K x in float64; reduces ||r||^2, sum(r) and sum(x); xc (or null)
// receives a copy of x, r32 (or null) the float32 copy of r.
__global__ void __launch_bounds__(kBlock) k_true_residual(LevelView<double> L, const double* __restrict__ f,
                                                         const double* __restrict__ x, double* __restrict__ r, int kper,
                                                         Reduce R, double* __restrict__ xc, float* __restrict__ r32)
{
    Tile t = tile(L.nx, L.ny, L.nz, kper);
    double acc[3] = {0.0, 0.0, 0.0};
    if (t.act) {
        for (int k = t.k0; k < t.k1; ++k) {
            const int c = cell(L.nx, L.ny, t.i, t.j, k);
            double s, d;
            nbsum<double>(L, t.i, t.j, k, c, [&](int m, int, int, int) { return x[m]; }, s, d);
            const double rv = f[c] - (d * x[c] - s);
            r[c] = rv;
            if (xc) xc[c] = x[c];
            if (r32) r32[c] = (float)rv;
            acc[0] += rv * rv;
            acc[1] += rv;
            acc[2] += x[c];
        }
    }
    reduce_finish<3>(acc, R);
}

// Reduces sum(x) over finite entries and the count of non-finite entries (and
// of entries <= 0 when check_pos).
__global__ void __launch_bounds__(kBlock) k_sum_check(int n, const double* __restrict__ x, int check_pos, Reduce R)
{
    double acc[2] = {0.0, 0.0};
    const int stride = gridDim.x * blockDim.x;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += stride) {
        const double v = x[c];
        const bool bad = !(v - v == 0.0) || (check_pos && !(v > 0.0));
        acc[0] += bad ? 0.0 : v;
        acc[1] += bad ? 1.0 : 0.0;
    }
    reduce_finish<2>(acc, R);
}

// y = a * (x - s[slot]/n) in float64, optionally reducing ||y||^2.
__global__ void __launch_bounds__(kBlock) k_shift_scale(int n, const double* __restrict__ x, double* __restrict__ y, double a,
                                                       Coefs mean, int want_red, Reduce R)
{
    const double m = mean.get();
    double acc[1] = {0.0};
    const int stride = gridDim.x * blockDim.x;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += stride) {
        const double v = a * (x[c] - m);
        y[c] = v;
        acc[0] += v * v;
    }
    if (want_red) reduce_finish<1>(acc, R);
}

// ---------------------------------------------------------------- set-up

// Finest-level face weights beta_f = 2/(rho_L + rho_R): IEEE division, zero on
// the wall faces, periodic in z.
__global__ void __launch_bounds__(kBlock) k_fine_faces(int nx, int ny, int nz, const double* __restrict__ rho,
                                                      double* __restrict__ wx, double* __restrict__ wy, double* __restrict__ wz,
                                                      int kper)
{
    Tile t = tile(nx, ny, nz, kper);
    if (!t.act) return;
    const int sy = nx, sz = nx * ny;
    for (int k = t.k0; k < t.k1; ++k) {
        const int c = cell(nx, ny, t.i, t.j, k);
        const int ct = k < nz - 1 ? c + sz : c - (nz - 1) * sz;
        const double rc = rho[c];
        wx[c] = t.i < nx - 1 ? 2.0 / (rc + rho[c + 1]) : 0.0;
        wy[c] = t.j < ny - 1 ? 2.0 / (rc + rho[c + sy]) : 0.0;
        wz[c] = 2.0 / (rc + rho[ct]);
    }
}

// The handle's copies of the density: float64 and, for a float32 preconditioner,
// float32 (one pass over the caller's array).
__global__ void __launch_bounds__(kBlock) k_take_density(int n, const double* __restrict__ rho, double* __restrict__ rho64,
                                                        float* __restrict__ rho32)
{
    const int stride = gridDim.x * blockDim.x;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += stride) {
        const double v = rho[c];
        rho64[c] = v;
        if (rho32) rho32[c] = (float)v;
    }
}

// 1/D of the finest level straight from the density, for the kernels that form
// their weights from it (no stored finest-level weights): D is the sum of
// beta_f = 2/(rho_L + rho_R) over the cell's faces, added in the order nbsum
// adds them, so the values equal those k_level_finish forms from k_fine_faces'
// weights, bit for bit.
__global__ void __launch_bounds__(kBlock) k_fine_diag(int nx, int ny, int nz, const double* __restrict__ rho,
                                                     double* __restrict__ invd64, float* __restrict__ invd32, int kper)
{
    Tile t = tile(nx, ny, nz, kper);
    if (!t.act) return;
    const int sy = nx, sz = nx * ny;
    for (int k = t.k0; k < t.k1; ++k) {
        const int c = cell(nx, ny, t.i, t.j, k);
        const int cb = k > 0 ? c - sz : c + (nz - 1) * sz, ct = k < nz - 1 ? c + sz : c - (nz - 1) * sz;
        const double r = rho[c];
        double d = 0.0;
        if (t.i > 0) d += 2.0 / (rho[c - 1] + r);
        if (t.i < nx - 1) d += 2.0 / (r + rho[c + 1]);
        if (t.j > 0) d += 2.0 / (rho[c - sy] + r);
        if (t.j < ny - 1) d += 2.0 / (r + rho[c + sy]);
        d += 2.0 / (rho[cb] + r);
        d += 2.0 / (r + rho[ct]);
        const double inv = 1.0 / d;
        if (invd64) invd64[c] = inv;
        if (invd32) invd32[c] = (float)inv;
    }
}

// The float32 1/D of the finest level for the float32 cycle, from the float32
// density, with the weights formed as its passes form them (2 / (rho_L + rho_R)
// by the hardware reciprocal), added in nbsum's order: the diagonal the float32
// passes' own weights imply (a float64 1/D would cost seven float64 divisions a
// cell for a value rounded to float32).
__global__ void __launch_bounds__(kBlock) k_fine_diag32(int nx, int ny, int nz, const float* __restrict__ rho,
                                                       float* __restrict__ invd32, int kper)
{
    Tile t = tile(nx, ny, nz, kper);
    if (!t.act) return;
    const int sy = nx, sz = nx * ny;
    auto beta = [](float a, float b) { return 2.0f * __builtin_amdgcn_rcpf(a + b); };
    for (int k = t.k0; k < t.k1; ++k) {
        const int c = cell(nx, ny, t.i, t.j, k);
        const int cb = k > 0 ? c - sz : c + (nz - 1) * sz, ct = k < nz - 1 ? c + sz : c - (nz - 1) * sz;
        const float r = rho[c];
        float d = 0.0f;
        if (t.i > 0) d += beta(rho[c - 1], r);
        if (t.i < nx - 1) d += beta(r, rho[c + 1]);
        if (t.j > 0) d += beta(rho[c - sy], r);
        if (t.j < ny - 1) d += beta(r, rho[c + sy]);
        d += beta(rho[cb], r);
        d += beta(r, rho[ct]);
        invd32[c] = __builtin_amdgcn_rcpf(d);
    }
}

// The first coarse level's face weights straight from the finest density: each
// is the sum of the four fine beta_f that form it, formed and added as
// k_fine_faces and k_coarsen form and add them (the same values, bit for bit).
__global__ void __launch_bounds__(kBlock) k_coarsen_rho(int nx, int ny, int nz, const double* __restrict__ rho, int cnx,
                                                       int cny, int cnz, double* __restrict__ wx, double* __restrict__ wy,
                                                       double* __restrict__ wz, int kper)
{
    Tile t = tile(cnx, cny, cnz, kper);
    if (!t.act) return;
    const int sy = nx, sz = nx * ny;
    for (int K = t.k0; K < t.k1; ++K) {
        double sx = 0.0, syw = 0.0, szw = 0.0;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                const int i = 2 * t.i + 1, j = 2 * t.j + a, k = 2 * K + b;
                const int c = cell(nx, ny, i, j, k);
                sx += i < nx - 1 ? 2.0 / (rho[c] + rho[c + 1]) : 0.0;
                const int cy = cell(nx, ny, 2 * t.i + a, 2 * t.j + 1, 2 * K + b);
                syw += 2 * t.j + 1 < ny - 1 ? 2.0 / (rho[cy] + rho[cy + sy]) : 0.0;
                const int kz = 2 * K + 1;
                const int cz = cell(nx, ny, 2 * t.i + a, 2 * t.j + b, kz);
                const int czt = kz < nz - 1 ? cz + sz : cz - (nz - 1) * sz;
                szw += 2.0 / (rho[cz] + rho[czt]);
            }
        const int cc = cell(cnx, cny, t.i, t.j, K);
        wx[cc] = sx;
        wy[cc] = syw;
        wz[cc] = szw;
    }
}

// The set-up passes over the finest density in one launch (density-formed
// finest weights, a coarse level below it): per coarse cell, for its 8 fine
// cells the handle's float64 and float32 copies of the density and 1/D (as
// k_fine_diag forms it with D64, else as k_fine_diag32 forms it), the first
// coarse level's face weights (as k_coarsen_rho forms them), and the count of
// density values that are not finite and > 0 (one value reduced).  Each fine
// value is formed from the same operands in the same order as by those
// kernels, so the results are the same bit for bit.
template <bool D64>
__global__ void __launch_bounds__(kBlock) k_fine_setup(int nx, int ny, int nz, const double* __restrict__ rho,
                                                      double* __restrict__ rho64, float* __restrict__ rho32,
                                                      double* __restrict__ invd64, float* __restrict__ invd32,
                                                      double* __restrict__ wx, double* __restrict__ wy,
                                                      double* __restrict__ wz, int kper, Reduce R)
{
    const int cnx = nx >> 1, cny = ny >> 1, cnz = nz >> 1;
    Tile t = tile(cnx, cny, cnz, kper);
    double acc[1] = {0.0};
    if (t.act) {
        const int i0 = 2 * t.i - 1, j0 = 2 * t.j - 1;  // fine index of v's slot 0 in x and y
        auto beta32 = [](float a, float b) { return 2.0f * __builtin_amdgcn_rcpf(a + b); };
        for (int K = t.k0; K < t.k1; ++K) {
            const int k0 = 2 * K - 1;
            // v[c][b][a]: the density at fine (i0 + a, j0 + b, k0 + c), a, b, c in 0..3, loaded for
            // the 2 x 2 x 2 cells of the coarse cell and their face neighbours (x and y clamped at
            // the walls, where the value is not used; z periodic)
            double v[4][4][4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int k = k0 + c < 0 ? k0 + c + nz : (k0 + c >= nz ? k0 + c - nz : k0 + c);
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int j = max(0, min(ny - 1, j0 + b));
#pragma unroll
                    for (int a = 0; a < 4; ++a) {
                        const int outside = (a == 0 || a == 3) + (b == 0 || b == 3) + (c == 0 || c == 3);
                        if (outside > 1) continue;
                        const int i = max(0, min(nx - 1, i0 + a));
                        v[c][b][a] = rho[cell(nx, ny, i, j, k)];
                    }
                }
            }
#pragma unroll
            for (int c = 1; c < 3; ++c) {
#pragma unroll
                for (int b = 1; b < 3; ++b) {
#pragma unroll
                    for (int a = 1; a < 3; ++a) {
                        const int i = i0 + a, j = j0 + b, k = k0 + c;
                        const int ci = cell(nx, ny, i, j, k);
                        const double r = v[c][b][a];
                        acc[0] += (!(r - r == 0.0) || !(r > 0.0)) ? 1.0 : 0.0;
                        rho64[ci] = r;
                        if (rho32) rho32[ci] = (float)r;
                        if constexpr (D64) {
                            double d = 0.0;
                            if (i > 0) d += 2.0 / (v[c][b][a - 1] + r);
                            if (i < nx - 1) d += 2.0 / (r + v[c][b][a + 1]);
                            if (j > 0) d += 2.0 / (v[c][b - 1][a] + r);
                            if (j < ny - 1) d += 2.0 / (r + v[c][b + 1][a]);
                            d += 2.0 / (v[c - 1][b][a] + r);
                            d += 2.0 / (r + v[c + 1][b][a]);
                            const double inv = 1.0 / d;
                            invd64[ci] = inv;
                            if (invd32) invd32[ci] = (float)inv;
                        } else {
                            const float rf = (float)r;
                            float d = 0.0f;
                            if (i > 0) d += beta32((float)v[c][b][a - 1], rf);
                            if (i < nx - 1) d += beta32(rf, (float)v[c][b][a + 1]);
                            if (j > 0) d += beta32((float)v[c][b - 1][a], rf);
                            if (j < ny - 1) d += beta32(rf, (float)v[c][b + 1][a]);
                            d += beta32((float)v[c - 1][b][a], rf);
                            d += beta32(rf, (float)v[c + 1][b][a]);
                            invd32[ci] = __builtin_amdgcn_rcpf(d);
                        }
                    }
                }
            }
            // coarse face weights: sums of the four fine beta_f across each face, in
            // k_coarsen_rho's order (a over y or x, b over z or y)
            double sx = 0.0, syw = 0.0, szw = 0.0;
#pragma unroll
            for (int a = 0; a < 2; ++a) {
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    sx += 2 * t.i + 1 < nx - 1 ? 2.0 / (v[b + 1][a + 1][2] + v[b + 1][a + 1][3]) : 0.0;
                    syw += 2 * t.j + 1 < ny - 1 ? 2.0 / (v[b + 1][2][a + 1] + v[b + 1][3][a + 1]) : 0.0;
                    szw += 2.0 / (v[2][b + 1][a + 1] + v[3][b + 1][a + 1]);
                }
            }
            const int cc = cell(cnx, cny, t.i, t.j, K);
            wx[cc] = sx;
            wy[cc] = syw;
            wz[cc] = szw;
        }
    }
    reduce_finish<1>(acc, R);
}

// Next coarse level: each coarse face weight is the sum of the four fine face
// weights that form it.
__global__ void __launch_bounds__(kBlock) k_coarsen(int nx, int ny, int nz, const double* __restrict__ fx,
                                                   const double* __restrict__ fy, const double* __restrict__ fz, int cnx, int cny,
                                                   int cnz, double* __restrict__ wx, double* __restrict__ wy,
                                                   double* __restrict__ wz, int kper)
{
    Tile t = tile(cnx, cny, cnz, kper);
    if (!t.act) return;
    for (int K = t.k0; K < t.k1; ++K) {
        double sx = 0.0, sy = 0.0, sz = 0.0;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                sx += fx[cell(nx, ny, 2 * t.i + 1, 2 * t.j + a, 2 * K + b)];
                sy += fy[cell(nx, ny, 2 * t.i + a, 2 * t.j + 1, 2 * K + b)];
                sz += fz[cell(nx, ny, 2 * t.i + a, 2 * t.j + b, 2 * K + 1)];
            }
        const int cc = cell(cnx, cny, t.i, t.j, K);
        wx[cc] = sx;
        wy[cc] = sy;
        wz[cc] = sz;
    }
}

// 1/D of a level plus float32 copies of its weights (when the float32 arrays
// exist) and bfloat16 copies (when those exist).
__global__ void __launch_bounds__(kBlock) k_level_finish(int nx, int ny, int nz, const double* __restrict__ wx,
                                                        const double* __restrict__ wy, const double* __restrict__ wz,
                                                        double* __restrict__ invd64, float* __restrict__ wx32,
                                                        float* __restrict__ wy32, float* __restrict__ wz32,
                                                        float* __restrict__ invd32, unsigned short* __restrict__ wx16,
                                                        unsigned short* __restrict__ wy16, unsigned short* __restrict__ wz16,
                                                        int kper)
{
    Tile t = tile(nx, ny, nz, kper);
    if (!t.act) return;
    LevelView<double> L{nx, ny, nz, wx, wy, wz, nullptr};
    for (int k = t.k0; k < t.k1; ++k) {
        const int c = cell(nx, ny, t.i, t.j, k);
        double s, d;
        nbsum<double>(L, t.i, t.j, k, c, [&](int, int, int, int) { return 0.0; }, s, d);
        const double inv = 1.0 / d;
        if (invd64) invd64[c] = inv;
        if (wx32) {
            wx32[c] = (float)wx[c];
            wy32[c] = (float)wy[c];
            wz32[c] = (float)wz[c];
            invd32[c] = (float)inv;
        }
        if (wx16) {
            wx16[c] = to_bf16((float)wx[c]);
            wy16[c] = to_bf16((float)wy[c]);
            wz16[c] = to_bf16((float)wz[c]);
        }
    }
}

// Dense inverse of K + (mean D / n) 1 1^T for the coarsest level (n <= kDenseRows;
// symmetric positive definite, so Gauss-Jordan elimination needs no pivoting).
// One block; thread t holds, in registers, kDenseSeg entries of row
// t / kDenseSegs: the columns s + kDenseSegs u (s = t mod kDenseSegs), so that
// the threads of a wavefront reading one u of the pivot row read consecutive
// words (distinct LDS banks).  The matrix is inverted in place: for each pivot
// p (with the old pivot row and column) a_pp <- 1 / a_pp, a_pj <- a_pj / a_pp,
// a_ip <- -a_ip / a_pp and a_ij <- a_ij - a_ip a_pj / a_pp elsewhere.  The pivot
// row and column are published in LDS by the threads that hold them,
// double-buffered: the holders of row and column p + 1 publish them as soon as
// step p has updated them, so each step takes one barrier.
constexpr int kDenseRows = 128;
constexpr int kDenseThreads = 1024;
constexpr int kDenseSeg = kDenseRows * kDenseRows / kDenseThreads;  // entries per thread
constexpr int kDenseSegs = kDenseRows / kDenseSeg;                  // threads per row
__global__ void __launch_bounds__(kDenseThreads) k_dense_inverse(int nx, int ny, int nz, const double* __restrict__ wx,
                                                                 const double* __restrict__ wy,
                                                                 const double* __restrict__ wz, double* __restrict__ M64,
                                                                 float* __restrict__ M32)
{
    const int n = nx * ny * nz;
    const int sy = nx, sz = nx * ny;
    __shared__ double diag[kDenseRows];
    __shared__ double prow[2][kDenseRows], pcol[2][kDenseRows];
    __shared__ double dmean;
    const int i = threadIdx.x / kDenseSegs, s0 = threadIdx.x % kDenseSegs;
    const bool own = i < n;
    auto col = [&](int u) { return s0 + kDenseSegs * u; };
    // cell i's neighbours and face weights, in the order the operator sums them
    int nb[6];
    double w[6];
    double d = 0.0;
    if (own) {
        const int ci = i % nx, cj = (i / nx) % ny, ck = i / sz;
        const int cb = ck > 0 ? i - sz : i + (nz - 1) * sz;
        const int ct = ck < nz - 1 ? i + sz : i - (nz - 1) * sz;
        nb[0] = ci > 0 ? i - 1 : -1;
        w[0] = ci > 0 ? wx[i - 1] : 0.0;
        nb[1] = ci < nx - 1 ? i + 1 : -1;
        w[1] = ci < nx - 1 ? wx[i] : 0.0;
        nb[2] = cj > 0 ? i - sy : -1;
        w[2] = cj > 0 ? wy[i - sy] : 0.0;
        nb[3] = cj < ny - 1 ? i + sy : -1;
        w[3] = cj < ny - 1 ? wy[i] : 0.0;
        nb[4] = cb;
        w[4] = wz[cb];
        nb[5] = ct;
        w[5] = wz[i];
#pragma unroll
        for (int f = 0; f < 6; ++f)
            if (nb[f] >= 0) d += w[f];
        if (s0 == 0) diag[i] = d;
    }
    __syncthreads();
    if (threadIdx.x == 0) {  // the mean diagonal, summed in cell order
        double sum = 0.0;
        for (int c = 0; c < n; ++c) sum += diag[c];
        dmean = sum / n;
    }
    __syncthreads();
    double a[kDenseSeg];
    const double base = dmean / n;
#pragma unroll
    for (int u = 0; u < kDenseSeg; ++u) a[u] = base;
    if (own) {
#pragma unroll
        for (int f = 0; f < 6; ++f) {
#pragma unroll
            for (int u = 0; u < kDenseSeg; ++u)
                if (nb[f] == col(u)) a[u] -= w[f];
        }
#pragma unroll
        for (int u = 0; u < kDenseSeg; ++u)
            if (i == col(u)) a[u] += d;
    }
    // row p and column p of the current matrix into LDS buffer buf (entries past
    // n are never read)
    auto publish = [&](int p, int buf) {
        if (p >= n) return;
        if (i == p) {
#pragma unroll
            for (int u = 0; u < kDenseSeg; ++u) prow[buf][col(u)] = a[u];
        }
        const int q = p / kDenseSegs;
        double v = a[0];
#pragma unroll
        for (int u = 1; u < kDenseSeg; ++u) v = (u == q) ? a[u] : v;
        if (s0 == p % kDenseSegs) pcol[buf][i] = v;
    };
    publish(0, 0);
    __syncthreads();
    for (int p = 0; p < n; ++p) {
        const int buf = p & 1;
        // every LDS read of the step is issued before any result is used (columns
        // past n read entries that are never written; their results are not stored)
        double pj[kDenseSeg];
#pragma unroll
        for (int u = 0; u < kDenseSeg; ++u) pj[u] = prow[buf][col(u)];
        const double piv = prow[buf][p];
        const double aip = pcol[buf][i];
        const double rp = 1.0 / piv;
        const double f = aip * rp;
        if (i == p) {
#pragma unroll
            for (int u = 0; u < kDenseSeg; ++u) a[u] = a[u] * rp;
        } else {
#pragma unroll
            for (int u = 0; u < kDenseSeg; ++u) a[u] = a[u] - f * pj[u];
        }
        if (s0 == p % kDenseSegs) {  // the entry in column p
            const int q = p / kDenseSegs;
            const double val = i == p ? rp : -f;
#pragma unroll
            for (int u = 0; u < kDenseSeg; ++u)
                if (u == q) a[u] = val;
        }
        publish(p + 1, buf ^ 1);
        __syncthreads();
    }
    if (own) {
#pragma unroll
        for (int u = 0; u < kDenseSeg; ++u) {
            if (col(u) < n) {
                M64[i * n + col(u)] = a[u];
                M32[i * n + col(u)] = (float)a[u];
            }
        }
    }
}

// ---------------------------------------------------------------- public element-wise operations

// rho = rho_l * (1 - a) + rho_g * a, rounded exactly as written (no contraction).
__global__ void __launch_bounds__(kBlock) k_density(size_t n, const double* __restrict__ a, double rho_l, double rho_g,
                                                   double* __restrict__ rho)
{
#pragma clang fp contract(off)
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += stride) {
        const double av = a[c];
        rho[c] = rho_l * (1.0 - av) + rho_g * av;
    }
}

// out = (((u_e - u_w) + (v_n - v_s)) + (w_t - w_b)) / (h*dt); wall faces carry zero.
// Each thread walks its z range carrying w of the plane below; u of the west
// cell comes from the lane before it, v of the south cell from the row below
// (LDS, one barrier per plane).  Threads outside the grid read clamped cells,
// take part in the exchanges and barriers, and store nothing.
__global__ void __launch_bounds__(kBlock) k_divergence(int nx, int ny, int nz, double hd, const double* __restrict__ u,
                                                      const double* __restrict__ v, const double* __restrict__ w,
                                                      double* __restrict__ out, int kper)
{
#pragma clang fp contract(off)
    __shared__ double sv[2][kBlock];  // v of each thread's cell, by plane parity
    const Tile t = tile(nx, ny, nz, kper);
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    const int sy = nx, sz = nx * ny;
    const int ic = min(t.i, nx - 1), jc = min(t.j, ny - 1);
    int c = cell(nx, ny, ic, jc, t.k0);
    double wb = w[t.k0 > 0 ? c - sz : c + (nz - 1) * sz];
    int par = 0;
    for (int k = t.k0; k < t.k1; ++k, c += sz, par ^= 1) {
        const double uc = u[c], vc = v[c], wc = w[c];
        double uw = __shfl_up(uc, 1, 64);
        if (threadIdx.x == 0) uw = ic > 0 ? u[c - 1] : 0.0;
        sv[par][tid] = vc;
        __syncthreads();
        double vs;
        if (threadIdx.y > 0) vs = sv[par][tid - blockDim.x];
        else vs = jc > 0 ? v[c - sy] : 0.0;
        const double ue = ic < nx - 1 ? uc : 0.0;
        const double vn = jc < ny - 1 ? vc : 0.0;
        if (t.act) out[c] = (((ue - uw) + (vn - vs)) + (wc - wb)) / hd;
        wb = wc;
    }
}

// out = A x = div(beta grad x) in float64 (the operator of step 11) from the
// stored finest-level face coefficients.
__global__ void __launch_bounds__(kBlock) k_apply_a(LevelView<double> L, double inv_h2, const double* __restrict__ x,
                                                   double* __restrict__ out, int kper)
{
    Tile t = tile(L.nx, L.ny, L.nz, kper);
    if (!t.act) return;
    for (int k = t.k0; k < t.k1; ++k) {
        const int c = cell(L.nx, L.ny, t.i, t.j, k);
        const double xc = x[c];
        double s, d;
        nbsum<double>(L, t.i, t.j, k, c, [&](int m, int, int, int) { return x[m] - xc; }, s, d);
        out[c] = s * inv_h2;
    }
}

// Projection on faces (step 12 restricted to face velocities), in place:
// u_f -= dt * beta_f * (p_R - p_L)/h; wall faces set to zero.  Each thread walks
// its z range carrying rho and p of the plane above into the next plane; rho
// and p of the east cell come from the lane after it, of the north cell from
// the row above (LDS, one barrier per plane).  Threads outside the grid read
// clamped cells, take part in the exchanges and barriers, and store nothing.
__global__ void __launch_bounds__(kBlock) k_project(int nx, int ny, int nz, double h, double dt, const double* __restrict__ rho,
                                                   const double* __restrict__ p, double* u, double* v, double* w, int kper)
{
#pragma clang fp contract(off)
    __shared__ double sr[2][kBlock], sp[2][kBlock];  // rho and p of each thread's cell, by plane parity
    const Tile t = tile(nx, ny, nz, kper);
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    const int sy = nx, sz = nx * ny;
    const int ic = min(t.i, nx - 1), jc = min(t.j, ny - 1);
    int c = cell(nx, ny, ic, jc, t.k0);
    double rc = rho[c], pc = p[c];
    int par = 0;
    for (int k = t.k0; k < t.k1; ++k, c += sz, par ^= 1) {
        const int ct = k < nz - 1 ? c + sz : c - (nz - 1) * sz;
        const double rt = rho[ct], pt = p[ct];
        double re = __shfl_down(rc, 1, 64), pe = __shfl_down(pc, 1, 64);
        if (threadIdx.x == blockDim.x - 1 && ic < nx - 1) {
            re = rho[c + 1];
            pe = p[c + 1];
        }
        sr[par][tid] = rc;
        sp[par][tid] = pc;
        __syncthreads();
        double rn = rc, pn = pc;
        if (threadIdx.y < blockDim.y - 1) {
            rn = sr[par][tid + blockDim.x];
            pn = sp[par][tid + blockDim.x];
        } else if (jc < ny - 1) {
            rn = rho[c + sy];
            pn = p[c + sy];
        }
        if (t.act) {
            u[c] = ic < nx - 1 ? u[c] - dt * ((2.0 / (rc + re)) * ((pe - pc) / h)) : 0.0;
            v[c] = jc < ny - 1 ? v[c] - dt * ((2.0 / (rc + rn)) * ((pn - pc) / h)) : 0.0;
            w[c] = w[c] - dt * ((2.0 / (rc + rt)) * ((pt - pc) / h));
        }
        rc = rt;
        pc = pt;
    }
}

// Step 12 of Section 2.2 on faces and cells in one pass, in place:
//   faces: u_f -= dt * beta_f (p_R - p_L)/h (wall faces set to zero), as k_project;
//   cells: u_c -= dt * (g_W + g_E)/2 per axis, g_f = beta_f (p_R - p_L)/h
//          [+ beta_f (pt_R - pt_L)/h], zero on the walls: the face-to-cell average
//          of the face pressure terms of p and (with PT) the surface-tension
//          pressure pt.
// Each thread walks its z range carrying rho, p, pt of the plane above and the
// top-face term into the next plane (as that plane's own values and bottom-face
// term: the same operands in the same order, so the same rounding).  A thread
// forms its cell's east and north faces; the west face term is the east term of
// the lane before it and the south term the north term of the row below (LDS,
// one barrier per plane).  East values come from the lane after it, north values
// from global memory (the row above is being read by the block).  Threads outside
// the grid read clamped cells, take part in the exchanges and barriers, and store
// nothing.
template <bool PT>
__global__ void __launch_bounds__(kBlock) k_correct_velocity(int nx, int ny, int nz, double h, double dt,
                                                            const double* __restrict__ rho, const double* __restrict__ p,
                                                            const double* __restrict__ pt, double* __restrict__ u,
                                                            double* __restrict__ v, double* __restrict__ w,
                                                            double* __restrict__ uc, double* __restrict__ vc,
                                                            double* __restrict__ wc, int kper)
{
#pragma clang fp contract(off)
    __shared__ double sgn[2][kBlock];  // north-face term of each thread's cell, by plane parity
    const Tile t = tile(nx, ny, nz, kper);
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    const int sy = nx, sz = nx * ny;
    const int ic = min(t.i, nx - 1), jc = min(t.j, ny - 1);
    const bool has_e = ic < nx - 1, has_n = jc < ny - 1, has_w = ic > 0, has_s = jc > 0;
    // face term of pressure q across the face between cells a (lower) and b (upper)
    auto term = [&](double beta, double qa, double qb) { return beta * ((qb - qa) / h); };
    int c = cell(nx, ny, ic, jc, t.k0);
    double rc = rho[c], pc = p[c], tc = PT ? pt[c] : 0.0;
    double gb;  // bottom-face term of the current plane
    {
        const int cb = t.k0 > 0 ? c - sz : c + (nz - 1) * sz;
        const double beta = 2.0 / (rho[cb] + rc);
        gb = term(beta, p[cb], pc);
        if (PT) gb = gb + term(beta, pt[cb], tc);
    }
    int par = 0;
    for (int k = t.k0; k < t.k1; ++k, c += sz, par ^= 1) {
        const int ct = k < nz - 1 ? c + sz : c - (nz - 1) * sz;
        const double rt = rho[ct], ptop = p[ct], ttop = PT ? pt[ct] : 0.0;
        // east neighbour: the lane after this one; the tile's last lane reads it
        double re = __shfl_down(rc, 1, 64), pe = __shfl_down(pc, 1, 64), te = PT ? __shfl_down(tc, 1, 64) : 0.0;
        if (threadIdx.x == blockDim.x - 1 && has_e) {
            re = rho[c + 1];
            pe = p[c + 1];
            if (PT) te = pt[c + 1];
        }
        const int cn = has_n ? c + sy : c;
        const double rn = rho[cn], pn = p[cn], tn = PT ? pt[cn] : 0.0;
        // east, north and top face: the p term (face projection) and the total term
        double ge_p = 0.0, gn_p = 0.0, ge = 0.0, gn = 0.0;
        if (has_e) {
            const double beta = 2.0 / (rc + re);
            ge_p = term(beta, pc, pe);
            ge = PT ? ge_p + term(beta, tc, te) : ge_p;
        }
        if (has_n) {
            const double beta = 2.0 / (rc + rn);
            gn_p = term(beta, pc, pn);
            gn = PT ? gn_p + term(beta, tc, tn) : gn_p;
        }
        const double beta_t = 2.0 / (rc + rt);
        const double gt_p = term(beta_t, pc, ptop);
        const double gt = PT ? gt_p + term(beta_t, tc, ttop) : gt_p;
        // west face: the east term of the lane before; the tile's first lane forms it
        double gw = __shfl_up(ge, 1, 64);
        if (threadIdx.x == 0) {
            gw = 0.0;
            if (has_w) {
                const double rw = rho[c - 1], beta = 2.0 / (rw + rc);
                gw = term(beta, p[c - 1], pc);
                if (PT) gw = gw + term(beta, pt[c - 1], tc);
            }
        }
        sgn[par][tid] = gn;
        __syncthreads();
        double gs;
        if (threadIdx.y > 0) {
            gs = sgn[par][tid - blockDim.x];
        } else {
            gs = 0.0;
            if (has_s) {
                const double rs = rho[c - sy], beta = 2.0 / (rs + rc);
                gs = term(beta, p[c - sy], pc);
                if (PT) gs = gs + term(beta, pt[c - sy], tc);
            }
        }
        if (t.act) {
            u[c] = has_e ? u[c] - dt * ge_p : 0.0;
            v[c] = has_n ? v[c] - dt * gn_p : 0.0;
            w[c] = w[c] - dt * gt_p;
            uc[c] = uc[c] - dt * (0.5 * (gw + ge));
            vc[c] = vc[c] - dt * (0.5 * (gs + gn));
            wc[c] = wc[c] - dt * (0.5 * (gb + gt));
        }
        gb = gt;
        rc = rt;
        pc = ptop;
        tc = ttop;
    }
}

// Right-hand side of the surface-tension pressure equation: out = div(beta f)
// with the face force f = sigma * (kappa_L + kappa_R)/2 * (a_R - a_L)/h, from
// the values at the face's lower (L) and upper (R) cell.
__device__ inline double st_flux(double rl, double rr, double al, double ar, double kl, double kr, double sigma, double h)
{
#pragma clang fp contract(off)
    const double beta = 2.0 / (rl + rr);
    const double f = sigma * (0.5 * (kl + kr)) * ((ar - al) / h);
    return beta * f;
}

// Each thread walks its z range: the cell's values and its top-face flux are
// carried into the next plane as that plane's own values and bottom-face flux
// (the same operands in the same order, so the same rounding).  In a plane each
// thread forms its east and north faces; the west face is the east face of the
// lane before it (same row of the tile) and the south face the north face of
// the row below it (through LDS), so a face shared by two cells of the tile is
// formed once.  Threads outside the grid read clamped cells, take part in the
// exchanges and barriers, and store nothing.
__global__ void __launch_bounds__(kBlock) k_surface_rhs(int nx, int ny, int nz, double h, double sigma,
                                                       const double* __restrict__ rho, const double* __restrict__ a,
                                                       const double* __restrict__ kap, double* __restrict__ out, int kper)
{
#pragma clang fp contract(off)
    __shared__ double sfn[2][kBlock];  // north-face flux of each thread's cell, by plane parity
    const Tile t = tile(nx, ny, nz, kper);
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    const int sy = nx, sz = nx * ny;
    const int ic = min(t.i, nx - 1), jc = min(t.j, ny - 1);
    int c = cell(nx, ny, ic, jc, t.k0);
    double rc = rho[c], ac = a[c], kc = kap[c];
    double fb;
    {
        const int cb = t.k0 > 0 ? c - sz : c + (nz - 1) * sz;
        fb = st_flux(rho[cb], rc, a[cb], ac, kap[cb], kc, sigma, h);
    }
    int par = 0;
    for (int k = t.k0; k < t.k1; ++k, c += sz, par ^= 1) {
        const int ct = k < nz - 1 ? c + sz : c - (nz - 1) * sz;
        const double rt = rho[ct], at = a[ct], kt = kap[ct];
        const double fe = ic < nx - 1 ? st_flux(rc, rho[c + 1], ac, a[c + 1], kc, kap[c + 1], sigma, h) : 0.0;
        const double fn = jc < ny - 1 ? st_flux(rc, rho[c + sy], ac, a[c + sy], kc, kap[c + sy], sigma, h) : 0.0;
        double fw = __shfl_up(fe, 1, 64);
        if (threadIdx.x == 0) fw = ic > 0 ? st_flux(rho[c - 1], rc, a[c - 1], ac, kap[c - 1], kc, sigma, h) : 0.0;
        sfn[par][tid] = fn;
        __syncthreads();
        double fs;
        if (threadIdx.y > 0) fs = sfn[par][tid - blockDim.x];
        else fs = jc > 0 ? st_flux(rho[c - sy], rc, a[c - sy], ac, kap[c - sy], kc, sigma, h) : 0.0;
        const double ft = st_flux(rc, rt, ac, at, kc, kt, sigma, h);
        if (t.act) out[c] = (((fe - fw) + (fn - fs)) + (ft - fb)) / h;
        fb = ft;
        rc = rt;
        ac = at;
        kc = kt;
    }
}

}  // namespace pp
