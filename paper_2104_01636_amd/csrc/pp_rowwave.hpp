// pp_rowwave.hpp -- row-wave plane-marching kernels (gfx950): the finest
// level's float64 passes and the passes of the coarse float32 levels with
// bfloat16 weights.
//
// The same operations as the march kernels of pp_march.hpp, laid out so that a
// wavefront covers one whole grid row: the level's x extent is 64 * CPT cells
// and lane l owns the CPT consecutive cells at l * CPT.  A block of 64 x BY
// threads is BY rows (one per wavefront) and walks a range of z planes.  (On
// the finest level a row of 128 or 256 cells can instead be split over WPR = 2
// wavefronts, a block of 64 WPR x BY threads; see march_rw.)
//   * x neighbours are in the lane's own registers or in the next / previous
//     lane (wavefront shifts); the walls at i = 0 and i = nx-1 bound every
//     row, so there is no x halo at all (on a tiled row every tile edge would
//     fetch a whole cache line for one element per array and plane);
//   * y neighbours of the block's inner rows come from a double-buffered LDS
//     copy of the plane (one barrier per plane), stored slot-major: cell e of
//     lane l at e * 64 + l, so that the wavefront's access to one slot is 64
//     consecutive elements and no two lanes meet in an LDS bank (lane-major,
//     l * CPT + e, put CPT lanes on each bank); the first and last row of the
//     block (whole wavefronts, so the branch is uniform) also load the row
//     beyond the tile, one full row per array;
//   * z neighbours come from a three-plane register queue, as in pp_march.hpp;
//   * each lane loads CPT consecutive elements per array and plane, which the
//     compiler issues as wide loads, and the loads of plane k+1 are in flight
//     while plane k is computed: several times the bytes in flight per wave of a
//     one-cell-per-lane march, which is what a bandwidth-bound pass needs.
// Face weights are formed from the density (finest level): beta_f = 2/(rho_L +
// rho_R), float64 by IEEE division (bit-equal to the set-up), float32 by the
// hardware reciprocal; a cell's west weight is its west neighbour's east weight
// and its bottom weight the top weight of the plane below, so a cell divides
// for its east, north, south and top faces only.
#pragma once
#include "pp_march.hpp"

namespace pp {

// Shifts of a value across the wavefront: lane l gets lane l+1's value
// (lane_next) or lane l-1's (lane_prev); the edge lane keeps its own.  DPP
// wave shifts (wave_shl:1 = 0x130, wave_shr:1 = 0x138) move 32 bits per VALU
// move without the LDS crossbar a bpermute takes; a double moves as two halves.
// Callers are in wavefront-uniform control flow (every lane active).
template <int CTRL>
__device__ inline int wave_shift32(int v)
{
    return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ inline float wave_shift(float v)
{
    return __int_as_float(wave_shift32<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ inline double wave_shift(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = wave_shift32<CTRL>((int)(b & 0xffffffffll));
    const int hi = wave_shift32<CTRL>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
template <class T>
__device__ inline T lane_next(T v) { return wave_shift<0x130>(v); }
template <class T>
__device__ inline T lane_prev(T v) { return wave_shift<0x138>(v); }

// Tile (row band and z range) of this block: grid.y bands of SY rows, grid.z
// z ranges, blocks dealt to the XCDs in contiguous runs (see tile_of_block).
__device__ inline void rw_tile(int& by, int& bz, int xcd)
{
    int bx;
    tile_of_block(bx, by, bz, xcd);
}

// One plane's global inputs of a row-wave lane: own raw inputs at k+1 (the
// plane above, for the z queue), apply's extras, and for the first / last
// wavefront of the block the raw inputs of the row beyond the tile; with
// density-formed weights (finest level) the density at k+1 and of the row
// beyond, with stored bfloat16 weights (coarse float32 levels) the cell's east,
// north and top weights and, for the first wavefront, the north weight of the
// row beyond (its south weight).
template <class T, int CPT, class Raw, class Ex>
struct RwRegs {
    Raw rn[CPT];   // raw inputs at (i, j, k+1)
    Ex ex[CPT];    // apply's extras at (i, j, k)
    T rho_n[CPT];  // density at (i, j, k+1)           | bfloat16 weights: top weight at (i, j, k)
    Raw rh[CPT];   // halo row raw inputs at (i, j +- 1, k)
    T rho_h[CPT];  // halo row density at (i, j +- 1, k) | bfloat16: north weight of row j - 1
    T w_e[CPT];    // bfloat16 weights: east and north weight at (i, j, k)
    T w_n[CPT];
};

// The row-wave march.  Op is the same interface as for march() (pp_march.hpp):
// load / val / extra / apply per cell; every lane calls apply for each of its
// cells at every plane (act false outside the grid).  WM: kWRho (weights from
// the density, finest level) or kWHalf (stored bfloat16 weights).  WPR: the
// wavefronts a row is split over (density weights only): lane l of the row
// (threadIdx.x) owns cells l * CPT ..; across the boundary between two of its
// wavefronts the x neighbour's value and density come from the row's LDS copy.
template <class T, int CPT, int BY, class Op, class Acc, int WM = kWRho, int WPR = 1>
__device__ inline void march_rw(const LevelView<T>& L, int kper, int xcd, Op& op, Acc& acc)
{
    static_assert(WM == kWRho || WM == kWHalf, "row-wave weights: density or bfloat16");
    static_assert(WPR == 1 || WM == kWRho, "split rows take their x neighbours' weights from the density");
    constexpr bool RHO = WM == kWRho;
    using Raw = typename Op::Raw;
    using Ex = typename Op::Ex;
    using Regs = RwRegs<T, CPT, Raw, Ex>;
    constexpr int NL = 64 * WPR;  // lanes per row
    constexpr int NX = NL * CPT;
    __shared__ T sv[2][BY][NX];   // stencil value of each cell, by plane parity (cell e of lane l at e * NL + l)
    __shared__ T sr[2][BY][NX];   // density (or north weight) of each cell, by plane parity
    const int lane = threadIdx.x, ty = threadIdx.y;
    const int wl = lane & 63, wr = lane >> 6;  // lane in its wavefront, wavefront in the row
    int by, bz;
    rw_tile(by, bz, xcd);
    const int j = by * BY + ty;
    const int k0 = bz * kper, k1 = min(L.nz, k0 + kper);
    if (k0 >= k1) return;  // an empty z range (none in the launches made here)
    const bool act = j < L.ny;
    const int jc = min(j, L.ny - 1);
    const int i0 = lane * CPT;
    const int sz = L.nx * L.ny;
    const int cbase = cell(L.nx, L.ny, i0, jc, 0);
    // the first and last wavefront of the block read the row beyond the tile
    const bool lo = ty == 0 && jc > 0, hi = ty == BY - 1 && jc < L.ny - 1;
    const int oj = lo ? -L.nx : (hi ? L.nx : 0);
    const bool in_n = j < L.ny - 1, in_s = j > 0;

    auto fetch = [&](Regs& S, int k) {
        const int c = cbase + k * sz;
        const int kt = k < L.nz - 1 ? k + 1 : 0;
        const int ct = c + (kt - k) * sz;
#pragma unroll
        for (int e = 0; e < CPT; ++e) {
            S.rn[e] = op.load(ct + e, i0 + e, jc, kt);
            S.ex[e] = op.extra(c + e);
            if constexpr (RHO) {
                S.rho_n[e] = L.rho[ct + e];
            } else {
                S.w_e[e] = (T)from_bf16(L.hwx[c + e]);
                S.w_n[e] = (T)from_bf16(L.hwy[c + e]);
                S.rho_n[e] = (T)from_bf16(L.hwz[c + e]);
            }
        }
        if (lo || hi) {
#pragma unroll
            for (int e = 0; e < CPT; ++e) {
                S.rh[e] = op.load(c + oj + e, i0 + e, jc + (lo ? -1 : 1), k);
                if constexpr (RHO) S.rho_h[e] = L.rho[c + oj + e];
                else S.rho_h[e] = lo ? (T)from_bf16(L.hwy[c + oj + e]) : T(0);
            }
        }
    };

    // prologue: values at the plane below the first and at the first
    const int kb0 = k0 > 0 ? k0 - 1 : L.nz - 1;
    T vm[CPT], vc[CPT], rho_c[CPT], wb[CPT];
    Raw rc[CPT];
    {
        const int c = cbase + k0 * sz, cb = cbase + kb0 * sz;
#pragma unroll
        for (int e = 0; e < CPT; ++e) {
            vm[e] = act ? op.val(op.load(cb + e, i0 + e, jc, kb0)) : T(0);
            rc[e] = op.load(c + e, i0 + e, jc, k0);
            vc[e] = act ? op.val(rc[e]) : T(0);
            if constexpr (RHO) {
                rho_c[e] = L.rho[c + e];
                wb[e] = face_beta(L.rho[cb + e], rho_c[e]);
            } else {
                rho_c[e] = T(0);
                wb[e] = (T)from_bf16(L.hwz[cb + e]);
            }
        }
    }
    Regs R[2];
    fetch(R[0], k0);

    auto step = [&](Regs& S, Regs& N, int k, int buf) {
        const int c = cbase + k * sz;
        if (k + 1 < k1) fetch(N, k + 1);
        T vp[CPT];
#pragma unroll
        for (int e = 0; e < CPT; ++e) {
            vp[e] = act ? op.val(S.rn[e]) : T(0);
            sv[buf][ty][e * NL + lane] = vc[e];
            if constexpr (RHO) sr[buf][ty][e * NL + lane] = act ? rho_c[e] : T(1);
            else sr[buf][ty][e * NL + lane] = act ? S.w_n[e] : T(0);
        }
        T vh[CPT];
        if (lo || hi) {
#pragma unroll
            for (int e = 0; e < CPT; ++e) vh[e] = op.val(S.rh[e]);
        }
        lds_barrier();
        // x neighbours: own registers, the previous lane's last cell, the next lane's first
        // (across a wavefront boundary of a split row: the row's LDS copy)
        T v_prev = lane_prev(vc[CPT - 1]), v_next = lane_next(vc[0]);
        if constexpr (WPR > 1) {
            if (wl == 0 && wr > 0) v_prev = sv[buf][ty][(CPT - 1) * NL + lane - 1];
            if (wl == 63 && wr < WPR - 1) v_next = sv[buf][ty][lane + 1];
        }
        T we[CPT];
        if constexpr (RHO) {
            T r_next = lane_next(rho_c[0]);
            if constexpr (WPR > 1) {
                if (wl == 63 && wr < WPR - 1) r_next = sr[buf][ty][lane + 1];
            }
#pragma unroll
            for (int e = 0; e < CPT; ++e) {
                const T re = e < CPT - 1 ? rho_c[e + 1] : r_next;
                we[e] = (i0 + e < NX - 1) ? face_beta(rho_c[e], re) : T(0);
            }
        } else {
#pragma unroll
            for (int e = 0; e < CPT; ++e) we[e] = S.w_e[e];  // zero on the wall face
        }
        T we_prev = lane_prev(we[CPT - 1]);
        if constexpr (WPR > 1) {  // the west neighbour's east weight, formed as it forms it
            if (wl == 0 && wr > 0) we_prev = face_beta(sr[buf][ty][(CPT - 1) * NL + lane - 1], rho_c[0]);
        }
#pragma unroll
        for (int e = 0; e < CPT; ++e) {
            const int i = i0 + e;
            const T vw = e > 0 ? vc[e - 1] : v_prev;
            const T ve = e < CPT - 1 ? vc[e + 1] : v_next;
            const T ww = e > 0 ? we[e - 1] : (i > 0 ? we_prev : T(0));
            T vs, vn, ws, wn, wt;
            if constexpr (RHO) {
                T rs, rn;
                if (ty > 0) { vs = sv[buf][ty - 1][e * NL + lane]; rs = sr[buf][ty - 1][e * NL + lane]; }
                else { vs = lo ? vh[e] : T(0); rs = lo ? S.rho_h[e] : T(1); }
                if (ty < BY - 1) { vn = sv[buf][ty + 1][e * NL + lane]; rn = sr[buf][ty + 1][e * NL + lane]; }
                else { vn = hi ? vh[e] : T(0); rn = hi ? S.rho_h[e] : T(1); }
                ws = in_s ? face_beta(rs, rho_c[e]) : T(0);
                wn = in_n ? face_beta(rho_c[e], rn) : T(0);
                wt = face_beta(rho_c[e], S.rho_n[e]);
            } else {
                if (ty > 0) { vs = sv[buf][ty - 1][e * NL + lane]; ws = sr[buf][ty - 1][e * NL + lane]; }
                else { vs = lo ? vh[e] : T(0); ws = lo ? S.rho_h[e] : T(0); }
                if (ty < BY - 1) vn = sv[buf][ty + 1][e * NL + lane];
                else vn = hi ? vh[e] : T(0);
                ws = in_s ? ws : T(0);
                wn = S.w_n[e];  // zero on the wall face
                wt = S.rho_n[e];
            }
            Stencil<T> st;
            st.s = ww * vw + we[e] * ve + ws * vs + wn * vn + wb[e] * vm[e] + wt * vp[e];
            st.d = ww + we[e] + ws + wn + wb[e] + wt;
            st.ww = ww;
            st.we = we[e];
            st.ws = ws;
            st.wn = wn;
            st.wb = wb[e];
            st.wt = wt;
            op.apply(c + e, i, j, k, vc[e], rc[e], S.ex[e], st, acc, act);
            wb[e] = wt;
        }
#pragma unroll
        for (int e = 0; e < CPT; ++e) {
            vm[e] = vc[e];
            vc[e] = vp[e];
            rc[e] = S.rn[e];
            if constexpr (RHO) rho_c[e] = S.rho_n[e];
        }
    };

    int k = k0;
    for (; k + 1 < k1; k += 2) {
        step(R[0], R[1], k, (k - k0) & 1);
        step(R[1], R[0], k + 1, (k + 1 - k0) & 1);
    }
    if (k < k1) step(R[0], R[1], k, (k - k0) & 1);
}

// Row-wave variants of the finest-level float64 passes of the Krylov step
// (same operations and reductions as m_dir_apply, m_true_residual, m_apply).
template <int CPT, int BY, class TZ, bool BETA, bool FINE, int WPR = 1>
__global__ void __launch_bounds__(64 * WPR * BY) r_dir_apply(LevelView<double> L, const TZ* __restrict__ z,
                                                      const double* __restrict__ dold, double* __restrict__ dnew,
                                                      double* __restrict__ q, const double* __restrict__ r,
                                                      double* __restrict__ x, Coefs beta, Coefs mean, int use_mean,
                                                      Coefs aprev, int kper, int xcd, Reduce R)
{
    OpDir<double, TZ, BETA, FINE> op{z, dold, r, dnew, q, x, BETA ? beta.get() : 0.0, use_mean ? mean.get() : 0.0,
                                     (FINE && BETA) ? aprev.get() : 0.0};
    constexpr int NV = FINE ? 1 : 2;
    double acc[NV] = {};
    march_rw<double, CPT, BY, decltype(op), double[NV], kWRho, WPR>(L, kper, xcd, op, acc);
    reduce_finish<NV>(acc, R);
}

template <int CPT, int BY, int WPR = 1>
__global__ void __launch_bounds__(64 * WPR * BY) r_true_residual(LevelView<double> L, const double* __restrict__ f,
                                                          const double* __restrict__ x, double* __restrict__ r, int kper,
                                                          int xcd, Reduce R, double* __restrict__ xc,
                                                          float* __restrict__ r32)
{
    OpResidual<double> op{f, x, r, xc, r32};
    double acc[3] = {0.0, 0.0, 0.0};
    march_rw<double, CPT, BY, decltype(op), double[3], kWRho, WPR>(L, kper, xcd, op, acc);
    reduce_finish<3>(acc, R);
}

template <int CPT, int BY, int WPR = 1>
__global__ void __launch_bounds__(64 * WPR * BY) r_apply(LevelView<double> L, const double* __restrict__ x,
                                                        double* __restrict__ y, double inv_h2, int kper, int xcd)
{
    OpApply<double> op{x, y, inv_h2};
    double acc[1] = {0.0};
    march_rw<double, CPT, BY, decltype(op), double[1], kWRho, WPR>(L, kper, xcd, op, acc);
}

// Row-wave passes of a float32 coarse level with stored bfloat16 weights (the
// float32 cycle's large coarse levels): the same operations as m_smooth_first,
// m_smooth_half, m_prolong_black and m_dir_apply there.
template <int CPT, int BY>
__global__ void __launch_bounds__(64 * BY) r_smooth_first(LevelView<float> L, const float* __restrict__ f,
                                                         float* __restrict__ x, int kper, int xcd, float omega)
{
    OpFirst<float> op{f, L.invd, x, omega};
    double acc[1] = {0.0};
    march_rw<float, CPT, BY, OpFirst<float>, double[1], kWHalf>(L, kper, xcd, op, acc);
}

template <int CPT, int BY, int NDOT, class TQ>
__global__ void __launch_bounds__(64 * BY) r_smooth_half(LevelView<float> L, const float* __restrict__ f, float* x,
                                                        int colour, int kper, int xcd, const TQ* __restrict__ q, Reduce R,
                                                        float omega)
{
    OpHalf<float, NDOT, TQ> op{f, x, q, colour, omega};
    double acc[NDOT > 0 ? NDOT : 1] = {};
    march_rw<float, CPT, BY, OpHalf<float, NDOT, TQ>, double[NDOT > 0 ? NDOT : 1], kWHalf>(L, kper, xcd, op, acc);
    if constexpr (NDOT > 0) reduce_finish<NDOT>(acc, R);
}

template <int CPT, int BY>
__global__ void __launch_bounds__(64 * BY) r_prolong_black(LevelView<float> L, const float* __restrict__ f,
                                                          const float* __restrict__ x, const float* __restrict__ e,
                                                          float wc, float* __restrict__ y, int kper, int xcd, float omega)
{
    OpProlongBlack<float> op{f, x, e, y, wc, omega, L.nx >> 1, L.ny >> 1};
    double acc[1] = {0.0};
    march_rw<float, CPT, BY, OpProlongBlack<float>, double[1], kWHalf>(L, kper, xcd, op, acc);
}

// XU: the K-cycle's deferred update of x (see OpDir), with coefficient aprev.
template <int CPT, int BY, bool BETA, int XU = 0>
__global__ void __launch_bounds__(64 * BY) r_dir_apply_f32(LevelView<float> L, const float* __restrict__ z,
                                                          const float* __restrict__ dold, float* __restrict__ dnew,
                                                          float* __restrict__ q, const float* __restrict__ r, Coefs beta,
                                                          Coefs mean, int use_mean, int kper, int xcd, Reduce R,
                                                          float* __restrict__ x = nullptr, Coefs aprev = Coefs{})
{
    using Op = OpDir<float, float, BETA, false, XU>;
    Op op{z, dold, r, dnew, q, x, BETA ? (float)beta.get() : 0.0f, use_mean ? (float)mean.get() : 0.0f,
          (BETA && XU > 0) ? (float)aprev.get() : 0.0f};
    double acc[2] = {0.0, 0.0};
    march_rw<float, CPT, BY, Op, double[2], kWHalf>(L, kper, xcd, op, acc);
    reduce_finish<2>(acc, R);
}

// The first sweep from zero of a K-cycle step on the step's residual r - alpha q
// of the previous step's r and q, which it also stores into fo.
template <int CPT, int BY>
__global__ void __launch_bounds__(64 * BY) r_smooth_first_r(LevelView<float> L, const float* __restrict__ r,
                                                           const float* __restrict__ q, Coefs alpha,
                                                           float* __restrict__ fo, float* __restrict__ x, int kper,
                                                           int xcd, float omega)
{
    OpFirstR<float> op{r, q, L.invd, fo, x, (float)alpha.get(), omega};
    double acc[1] = {0.0};
    march_rw<float, CPT, BY, OpFirstR<float>, double[1], kWHalf>(L, kper, xcd, op, acc);
}

}  // namespace pp
