// pp_rowfused.hpp -- row-wave forms of the two fused float32 passes of the
// finest level (gfx950): the first red-black sweep from a zero guess with the
// restriction of its residual, and the prolongation with the black update and
// the red half-sweep after it.
//
// Layout as in pp_rowwave.hpp: a wavefront is one whole grid row (lane l owns
// the CPT consecutive cells at l * CPT), a block is BY rows and walks a z range.
// Both passes need values two cells away (a red cell's residual needs its black
// neighbours' new values, which need their red neighbours), so the block's
// first and last row are a ring computed again by the neighbouring blocks, the
// march runs one plane below and one above the block's range, and the second
// stage trails the first by one plane.  Rows span the whole x extent (walls at
// both ends), so there is no ring and no halo in x: x neighbours are in the
// lane's registers or the next / previous lane (shuffles), y neighbours in a
// double-buffered LDS copy of the plane (one barrier per plane; slot-major,
// cell e of lane l at e * 64 + l, free of bank conflicts), z neighbours in
// registers.  The ring rows also load the row beyond the tile.
//
// The first pass uses the red-black structure to halve its second stage: a
// black cell updated from zero, x = omega (s + f) / D with s the sum over its
// red neighbours, leaves the residual f - K x = (1 - omega) (s + f) (zero for
// Gauss-Seidel), known after the first stage; a red cell, x = omega f / D,
// leaves (1 - omega) f + (sum over its black neighbours' new values).  So only
// red cells need a second stencil.  D is the diagonal the first stage divides
// by (the stored float32 1/D of the level), so these identities hold up to the
// rounding of D against the density-formed weights (about 1e-7 relative), an
// approximation the preconditioner absorbs.
#pragma once
#include "pp_rowwave.hpp"

namespace pp {

// Row-wave first sweep from zero + residual restriction (replaces m_first_restrict):
// x = red omega f/D, black x + omega ((s + f)/D - x) from zero; rc = sum of the
// residual over the 8 children of each coarse cell.  CPT even (x pairs of the
// restriction are inside a lane), real planes per block even (z pairs).
template <int CPT, int BY>
__global__ void __launch_bounds__(64 * BY) r_first_restrict(LevelView<float> L, const float* __restrict__ f,
                                                           float* __restrict__ x, float* __restrict__ rc, int kper,
                                                           int xcd, float omega)
{
    static_assert(CPT % 2 == 0, "x pairs of the restriction lie inside a lane");
    constexpr int NX = 64 * CPT, SY = BY - 2, HP = CPT / 2;
    __shared__ float s_val[2][BY][NX];  // red value omega f/D of each cell, by plane parity
    __shared__ float s_rho[2][BY][NX];  // density, by plane parity
    __shared__ float s_x[2][BY][NX];    // new x of each cell, by plane parity (read one plane later)
    __shared__ float s_r[BY][NX / 2];   // x-pair sums of the residual of a plane pair, by row
    const float* __restrict__ invd = L.invd;
    const float* __restrict__ rho = L.rho;
    const int lane = threadIdx.x, ty = threadIdx.y;
    int by, bz;
    rw_tile(by, bz, xcd);
    const int j = by * SY + ty - 1;  // rows 0 and BY-1 of the block are the ring
    const int k0 = bz * kper, k1 = min(L.nz, k0 + kper);
    if (k0 >= k1) return;  // an empty z range (none in the launches made here)
    const bool act = j >= 0 && j < L.ny;
    const bool own = act && ty >= 1 && ty <= BY - 2;
    const int jc = max(0, min(j, L.ny - 1));
    const int i0 = lane * CPT;
    const int sz = L.nx * L.ny;
    const int cbase = cell(L.nx, L.ny, i0, jc, 0);
    const bool lo = ty == 0 && act && j > 0, hi = ty == BY - 1 && act && j < L.ny - 1;
    const int oj = lo ? -L.nx : (hi ? L.nx : 0);
    const bool in_n = j < L.ny - 1, in_s = j > 0;
    const int cnx = L.nx >> 1, cny = L.ny >> 1;
    auto plane = [&](int v) { return v < 0 ? v + L.nz : (v >= L.nz ? v - L.nz : v); };

    struct In {
        float f[CPT], d[CPT], r[CPT];     // f, 1/D and density at plane k+1 (own row)
        float fh[CPT], dh[CPT], rh[CPT];  // f, 1/D and density at plane k (row beyond the tile)
    };
    auto fetch = [&](In& S, int k) {
        const int kt = k < L.nz - 1 ? k + 1 : 0;
        const int ct = cbase + kt * sz;
#pragma unroll
        for (int e = 0; e < CPT; ++e) {
            S.f[e] = f[ct + e];
            S.d[e] = invd[ct + e];
            S.r[e] = rho[ct + e];
        }
        if (lo || hi) {
            const int ch = cbase + k * sz + oj;
#pragma unroll
            for (int e = 0; e < CPT; ++e) {
                S.fh[e] = f[ch + e];
                S.dh[e] = invd[ch + e];
                S.rh[e] = rho[ch + e];
            }
        }
    };

    // plane k of the march: red values (vm below, vc current), f and 1/D, density,
    // bottom weights; second stage: x of the two planes below, f and the weights
    // of the red cells of the plane below
    const int vlo = k0 - 1, vhi = k1 + 1;
    float vm[CPT], vc[CPT], fc[CPT], dc[CPT], rho_c[CPT], wb[CPT];
    {
        const int ks = plane(vlo), kb = plane(vlo - 1);
        const int c = cbase + ks * sz, cb = cbase + kb * sz;
#pragma unroll
        for (int e = 0; e < CPT; ++e) {
            vm[e] = act ? omega * (f[cb + e] * invd[cb + e]) : 0.0f;
            fc[e] = f[c + e];
            dc[e] = invd[c + e];
            vc[e] = act ? omega * (fc[e] * dc[e]) : 0.0f;
            rho_c[e] = rho[c + e];
            wb[e] = face_beta(rho[cb + e], rho_c[e]);
        }
    }
    float xm2[CPT] = {}, xm1[CPT] = {};  // new x at the planes two and one below
    float rm1[CPT] = {};                 // residual of the black cells one plane below
    float fr[HP], ws6[HP][6];            // red cells one plane below: f and weights w, e, s, n, b, t
    float part[HP] = {}, pend[HP] = {};  // z-pair partial sums; the row pair's sum awaiting its partner row
    int pend_k = -1;                     // coarse plane of pend (-1: nothing pending)
    In R[2];
    fetch(R[0], plane(vlo));

    auto step = [&](In& S, In& N, int v, int buf) {
        const int k = plane(v);
        const int c = cbase + k * sz;
        if (v + 1 < vhi) fetch(N, plane(v + 1));
        float vp[CPT], vh[CPT];
#pragma unroll
        for (int e = 0; e < CPT; ++e) {
            vp[e] = act ? omega * (S.f[e] * S.d[e]) : 0.0f;
            s_val[buf][ty][e * 64 + lane] = vc[e];
            s_rho[buf][ty][e * 64 + lane] = act ? rho_c[e] : 1.0f;
        }
        if (lo || hi) {
#pragma unroll
            for (int e = 0; e < CPT; ++e) vh[e] = omega * (S.fh[e] * S.dh[e]);
        }
        lds_barrier();
        // a row pair's restriction sum left by the previous plane: rows ty odd add row ty+1
        if (pend_k >= 0) {
            if ((ty & 1) && own && j + 1 < L.ny) {
#pragma unroll
                for (int h = 0; h < HP; ++h) pend[h] += s_r[ty + 1][h * 64 + lane];
            }
            if ((ty & 1) && own) {
                float* dst = rc + cell(cnx, cny, lane * HP, j >> 1, pend_k);
#pragma unroll
                for (int h = 0; h < HP; ++h) dst[h] = pend[h];
            }
            pend_k = -1;
        }
        // first stage at plane k: weights from the density, red cells their value,
        // black cells one SOR update from their red neighbours
        const float v_prev = lane_prev(vc[CPT - 1]), v_next = lane_next(vc[0]);
        const float r_next = lane_next(rho_c[0]);
        float we[CPT];
#pragma unroll
        for (int e = 0; e < CPT; ++e) {
            const float re = e < CPT - 1 ? rho_c[e + 1] : r_next;
            we[e] = (i0 + e < NX - 1) ? face_beta(rho_c[e], re) : 0.0f;
        }
        const float we_prev = lane_prev(we[CPT - 1]);
        float x1[CPT], rb[CPT];
        float wsv[CPT][6];
#pragma unroll
        for (int e = 0; e < CPT; ++e) {
            const int i = i0 + e;
            const float vw = e > 0 ? vc[e - 1] : v_prev;
            const float ve = e < CPT - 1 ? vc[e + 1] : v_next;
            const float ww = e > 0 ? we[e - 1] : (i > 0 ? we_prev : 0.0f);
            float vs, vn, rs, rn;
            if (ty > 0) { vs = s_val[buf][ty - 1][e * 64 + lane]; rs = s_rho[buf][ty - 1][e * 64 + lane]; }
            else { vs = lo ? vh[e] : 0.0f; rs = lo ? S.rh[e] : 1.0f; }
            if (ty < BY - 1) { vn = s_val[buf][ty + 1][e * 64 + lane]; rn = s_rho[buf][ty + 1][e * 64 + lane]; }
            else { vn = hi ? vh[e] : 0.0f; rn = hi ? S.rh[e] : 1.0f; }
            const float ws = in_s ? face_beta(rs, rho_c[e]) : 0.0f;
            const float wn = in_n ? face_beta(rho_c[e], rn) : 0.0f;
            const float wt = face_beta(rho_c[e], S.r[e]);
            wsv[e][0] = ww; wsv[e][1] = we[e]; wsv[e][2] = ws; wsv[e][3] = wn; wsv[e][4] = wb[e]; wsv[e][5] = wt;
            const bool red = ((i + j + k) & 1) == 0;
            if (red) {
                x1[e] = act ? vc[e] : 0.0f;
                rb[e] = 0.0f;
            } else {
                const float s = ww * vw + we[e] * ve + ws * vs + wn * vn + wb[e] * vm[e] + wt * vp[e];
                const float sf = s + fc[e];
                x1[e] = act ? omega * (sf * dc[e]) : 0.0f;
                rb[e] = (1.0f - omega) * sf;  // f - K x of the black cell (x from zero: D x = omega sf)
            }
            wb[e] = wt;
        }
        // write x of the block's own cells at its real planes; keep it for the next plane's second stage
        const bool real = v >= k0 && v < k1;
        if (own && real) {
#pragma unroll
            for (int e = 0; e < CPT; ++e) x[c + e] = x1[e];
        }
#pragma unroll
        for (int e = 0; e < CPT; ++e) s_x[buf][ty][e * 64 + lane] = x1[e];
        // second stage at plane k-1 (a real plane from v = k0 + 1 on): residual of its red cells
        // from the new x of their black neighbours, then the restriction
        if (v >= k0 + 1) {
            const int km = plane(v - 1);
            const int bm = buf ^ 1;
            const float x_prev = lane_prev(xm1[CPT - 1]), x_next = lane_next(xm1[0]);
            float r[CPT];
#pragma unroll
            for (int e = 0; e < CPT; ++e) {
                const int i = i0 + e;
                const bool red = ((i + j + km) & 1) == 0;
                if (red) {
                    // neighbours of a red cell are black
                    const int hh = e >> 1;
                    const float xw = e > 0 ? xm1[e - 1] : x_prev;
                    const float xe = e < CPT - 1 ? xm1[e + 1] : x_next;
                    const float xs = ty > 0 ? s_x[bm][ty - 1][e * 64 + lane] : 0.0f;
                    const float xn = ty < BY - 1 ? s_x[bm][ty + 1][e * 64 + lane] : 0.0f;
                    const float s = ws6[hh][0] * xw + ws6[hh][1] * xe + ws6[hh][2] * xs + ws6[hh][3] * xn +
                                    ws6[hh][4] * xm2[e] + ws6[hh][5] * x1[e];
                    r[e] = (1.0f - omega) * fr[hh] + s;
                } else {
                    r[e] = rm1[e];
                }
            }
            float p[HP];
#pragma unroll
            for (int q = 0; q < HP; ++q) p[q] = own ? r[2 * q] + r[2 * q + 1] : 0.0f;
            if (((v - 1 - k0) & 1) == 0) {
#pragma unroll
                for (int q = 0; q < HP; ++q) part[q] = p[q];
            } else {
                // second plane of the pair: rows ty even hand their sum to row ty-1 (next plane)
#pragma unroll
                for (int q = 0; q < HP; ++q) pend[q] = part[q] + p[q];
                if (!(ty & 1)) {
#pragma unroll
                    for (int q = 0; q < HP; ++q) s_r[ty][q * 64 + lane] = pend[q];
                }
                pend_k = km >> 1;
            }
        }
        // shift the queues; keep the red cells' f and weights of plane k for the next second stage
#pragma unroll
        for (int e = 0; e < CPT; ++e) {
            const bool red = ((i0 + e + j + k) & 1) == 0;
            if (red) {
                const int hh = e >> 1;
                fr[hh] = fc[e];
#pragma unroll
                for (int w = 0; w < 6; ++w) ws6[hh][w] = wsv[e][w];
            }
            rm1[e] = rb[e];
            xm2[e] = xm1[e];
            xm1[e] = x1[e];
            vm[e] = vc[e];
            vc[e] = vp[e];
            fc[e] = S.f[e];
            dc[e] = S.d[e];
            rho_c[e] = S.r[e];
        }
    };

    int v = vlo;
    for (; v + 1 < vhi; v += 2) {
        step(R[0], R[1], v, (v - vlo) & 1);
        step(R[1], R[0], v + 1, (v + 1 - vlo) & 1);
    }
    if (v < vhi) step(R[0], R[1], v, (v - vlo) & 1);
    // the last row pair's sum
    if (pend_k >= 0) {
        lds_barrier();
        if ((ty & 1) && own) {
            if (j + 1 < L.ny) {
#pragma unroll
                for (int h = 0; h < HP; ++h) pend[h] += s_r[ty + 1][h * 64 + lane];
            }
            float* dst = rc + cell(cnx, cny, lane * HP, j >> 1, pend_k);
#pragma unroll
            for (int h = 0; h < HP; ++h) dst[h] = pend[h];
        }
    }
}

// Row-wave prolongation, black update and red half-sweep (replaces m_prolong_half):
// y = x + wc P e on red cells, black cells one SOR update from them, then one
// plane behind the red cells one SOR update from their black neighbours'
// new values: z (black cells keep y).  NDOT dots over the block's own cells:
// sum(z), <z, q>, <z, f> and sum(f).  CPT even (the parents of a lane's cells are whole).
template <int CPT, int BY, int NDOT, class TQ>
__global__ void __launch_bounds__(64 * BY) r_prolong_half(LevelView<float> L, const float* __restrict__ f,
                                                         const float* __restrict__ x, const float* __restrict__ ec,
                                                         float wc, float* __restrict__ z, const TQ* __restrict__ q,
                                                         Reduce R, int kper, int xcd, float omega)
{
    static_assert(CPT % 2 == 0, "a lane's cells have whole parents");
    constexpr int NX = 64 * CPT, SY = BY - 2, HP = CPT / 2;
    __shared__ float s_val[2][BY][NX];  // prolongated value x + wc P e of each cell, by plane parity
    __shared__ float s_rho[2][BY][NX];  // density, by plane parity
    __shared__ float s_y[2][BY][NX];    // y after the black update, by plane parity (read one plane later)
    const float* __restrict__ rho = L.rho;
    const int lane = threadIdx.x, ty = threadIdx.y;
    int by, bz;
    rw_tile(by, bz, xcd);
    const int j = by * SY + ty - 1;
    const int k0 = bz * kper, k1 = min(L.nz, k0 + kper);
    if (k0 >= k1) {  // an empty z range (none in the launches made here): a zero partial
        if constexpr (NDOT > 0) {
            double zero[NDOT] = {};
            reduce_finish<NDOT>(zero, R);
        }
        return;
    }
    const bool act = j >= 0 && j < L.ny;
    const bool own = act && ty >= 1 && ty <= BY - 2;
    const int jc = max(0, min(j, L.ny - 1));
    const int i0 = lane * CPT;
    const int sz = L.nx * L.ny;
    const int cbase = cell(L.nx, L.ny, i0, jc, 0);
    const bool lo = ty == 0 && act && j > 0, hi = ty == BY - 1 && act && j < L.ny - 1;
    const int jh = jc + (lo ? -1 : (hi ? 1 : 0));
    const bool in_n = j < L.ny - 1, in_s = j > 0;
    const int cnx = L.nx >> 1, cny = L.ny >> 1;
    auto plane = [&](int v) { return v < 0 ? v + L.nz : (v >= L.nz ? v - L.nz : v); };
    // parents of the lane's cells in row jj of plane k: coarse cells lane*HP .. lane*HP + HP-1
    auto parent = [&](int jj, int k) { return cell(cnx, cny, lane * HP, jj >> 1, k >> 1); };

    struct In {
        float x[CPT], e[HP], r[CPT], f[CPT];  // own row at plane k+1: x, parents, density, f
        float xh[CPT], eh[HP], rh[CPT];       // the row beyond the tile at plane k
        TQ q[CPT];                            // q at plane k-1 (the second stage's plane)
    };
    auto fetch = [&](In& S, int v) {
        const int k = plane(v), kt = plane(v + 1);
        const int ct = cbase + kt * sz, pt = parent(jc, kt);
#pragma unroll
        for (int e = 0; e < CPT; ++e) {
            S.x[e] = x[ct + e];
            S.r[e] = rho[ct + e];
            S.f[e] = f[ct + e];
        }
#pragma unroll
        for (int h = 0; h < HP; ++h) S.e[h] = ec[pt + h];
        if (lo || hi) {
            const int ch = cell(L.nx, L.ny, i0, jh, k), ph = parent(jh, k);
#pragma unroll
            for (int e = 0; e < CPT; ++e) {
                S.xh[e] = x[ch + e];
                S.rh[e] = rho[ch + e];
            }
#pragma unroll
            for (int h = 0; h < HP; ++h) S.eh[h] = ec[ph + h];
        }
        if constexpr (NDOT >= 2) {
            const int cq = cbase + plane(v - 1) * sz;
#pragma unroll
            for (int e = 0; e < CPT; ++e) S.q[e] = q[cq + e];
        }
    };

    const int vlo = k0 - 1, vhi = k1 + 1;
    float vm[CPT], vc[CPT], fc[CPT], rho_c[CPT], wb[CPT];
    {
        const int ks = plane(vlo), kb = plane(vlo - 1);
        const int c = cbase + ks * sz, cb = cbase + kb * sz;
        const int p0 = parent(jc, ks), pb = parent(jc, kb);
#pragma unroll
        for (int e = 0; e < CPT; ++e) {
            vm[e] = act ? x[cb + e] + wc * ec[pb + (e >> 1)] : 0.0f;
            vc[e] = act ? x[c + e] + wc * ec[p0 + (e >> 1)] : 0.0f;
            fc[e] = f[c + e];
            rho_c[e] = rho[c + e];
            wb[e] = face_beta(rho[cb + e], rho_c[e]);
        }
    }
    float ym2[CPT] = {}, ym1[CPT] = {};  // y at the planes two and one below
    float fr[HP], ws6[HP][6];            // red cells one plane below: f and weights w, e, s, n, b, t
    float fm1[CPT] = {};                 // f one plane below (NDOT >= 3)
    double acc[NDOT > 0 ? NDOT : 1] = {};
    In Rg[2];
    fetch(Rg[0], vlo);

    auto step = [&](In& S, In& N, int v, int buf) {
        const int k = plane(v);
        if (v + 1 < vhi) fetch(N, v + 1);
        float vp[CPT], vh[CPT];
#pragma unroll
        for (int e = 0; e < CPT; ++e) {
            vp[e] = act ? S.x[e] + wc * S.e[e >> 1] : 0.0f;
            s_val[buf][ty][e * 64 + lane] = vc[e];
            s_rho[buf][ty][e * 64 + lane] = act ? rho_c[e] : 1.0f;
        }
        if (lo || hi) {
#pragma unroll
            for (int e = 0; e < CPT; ++e) vh[e] = S.xh[e] + wc * S.eh[e >> 1];
        }
        lds_barrier();
        // first stage at plane k: red cells take the prolongated value, black cells one
        // SOR update from their red neighbours
        const float v_prev = lane_prev(vc[CPT - 1]), v_next = lane_next(vc[0]);
        const float r_next = lane_next(rho_c[0]);
        float we[CPT];
#pragma unroll
        for (int e = 0; e < CPT; ++e) {
            const float re = e < CPT - 1 ? rho_c[e + 1] : r_next;
            we[e] = (i0 + e < NX - 1) ? face_beta(rho_c[e], re) : 0.0f;
        }
        const float we_prev = lane_prev(we[CPT - 1]);
        float y1[CPT];
        float wsv[CPT][6];
#pragma unroll
        for (int e = 0; e < CPT; ++e) {
            const int i = i0 + e;
            const float vw = e > 0 ? vc[e - 1] : v_prev;
            const float ve = e < CPT - 1 ? vc[e + 1] : v_next;
            const float ww = e > 0 ? we[e - 1] : (i > 0 ? we_prev : 0.0f);
            float vs, vn, rs, rn;
            if (ty > 0) { vs = s_val[buf][ty - 1][e * 64 + lane]; rs = s_rho[buf][ty - 1][e * 64 + lane]; }
            else { vs = lo ? vh[e] : 0.0f; rs = lo ? S.rh[e] : 1.0f; }
            if (ty < BY - 1) { vn = s_val[buf][ty + 1][e * 64 + lane]; rn = s_rho[buf][ty + 1][e * 64 + lane]; }
            else { vn = hi ? vh[e] : 0.0f; rn = hi ? S.rh[e] : 1.0f; }
            const float ws = in_s ? face_beta(rs, rho_c[e]) : 0.0f;
            const float wn = in_n ? face_beta(rho_c[e], rn) : 0.0f;
            const float wt = face_beta(rho_c[e], S.r[e]);
            wsv[e][0] = ww; wsv[e][1] = we[e]; wsv[e][2] = ws; wsv[e][3] = wn; wsv[e][4] = wb[e]; wsv[e][5] = wt;
            const bool red = ((i + j + k) & 1) == 0;
            float yv = vc[e];
            if (!red && act) {
                const float s = ww * vw + we[e] * ve + ws * vs + wn * vn + wb[e] * vm[e] + wt * vp[e];
                const float d = ww + we[e] + ws + wn + wb[e] + wt;
                yv = gs_value(s, fc[e], d);
                if (omega != 1.0f) yv = vc[e] + omega * (yv - vc[e]);
            }
            y1[e] = act ? yv : 0.0f;
            wb[e] = wt;
        }
#pragma unroll
        for (int e = 0; e < CPT; ++e) s_y[buf][ty][e * 64 + lane] = y1[e];
        // second stage at plane k-1 (real from v = k0 + 1 on): red cells one SOR update from
        // their black neighbours' y; write z and reduce the dots
        if (v >= k0 + 1) {
            const int km = plane(v - 1);
            const int bm = buf ^ 1;
            const float y_prev = lane_prev(ym1[CPT - 1]), y_next = lane_next(ym1[0]);
            float zv[CPT];
#pragma unroll
            for (int e = 0; e < CPT; ++e) {
                const int i = i0 + e;
                const bool red = ((i + j + km) & 1) == 0;
                zv[e] = ym1[e];
                if (red) {
                    const int hh = e >> 1;
                    const float yw = e > 0 ? ym1[e - 1] : y_prev;
                    const float ye = e < CPT - 1 ? ym1[e + 1] : y_next;
                    const float ys = ty > 0 ? s_y[bm][ty - 1][e * 64 + lane] : 0.0f;
                    const float yn = ty < BY - 1 ? s_y[bm][ty + 1][e * 64 + lane] : 0.0f;
                    const float s = ws6[hh][0] * yw + ws6[hh][1] * ye + ws6[hh][2] * ys + ws6[hh][3] * yn +
                                    ws6[hh][4] * ym2[e] + ws6[hh][5] * y1[e];
                    const float d = ws6[hh][0] + ws6[hh][1] + ws6[hh][2] + ws6[hh][3] + ws6[hh][4] + ws6[hh][5];
                    float t = gs_value(s, fr[hh], d);
                    if (omega != 1.0f) t = ym1[e] + omega * (t - ym1[e]);
                    zv[e] = t;
                }
            }
            if (own) {
                const int cm = cbase + km * sz;
#pragma unroll
                for (int e = 0; e < CPT; ++e) {
                    z[cm + e] = zv[e];
                    if constexpr (NDOT >= 1) acc[0] += (double)zv[e];
                    if constexpr (NDOT >= 2) acc[1] += (double)zv[e] * (double)S.q[e];
                    if constexpr (NDOT >= 3) acc[2] += (double)zv[e] * (double)fm1[e];
                    if constexpr (NDOT >= 4) acc[3] += (double)fm1[e];
                }
            }
        }
#pragma unroll
        for (int e = 0; e < CPT; ++e) {
            const bool red = ((i0 + e + j + k) & 1) == 0;
            if (red) {
                const int hh = e >> 1;
                fr[hh] = fc[e];
#pragma unroll
                for (int w = 0; w < 6; ++w) ws6[hh][w] = wsv[e][w];
            }
            ym2[e] = ym1[e];
            ym1[e] = y1[e];
            vm[e] = vc[e];
            vc[e] = vp[e];
            if constexpr (NDOT >= 3) fm1[e] = fc[e];
            fc[e] = S.f[e];
            rho_c[e] = S.r[e];
        }
    };

    int v = vlo;
    for (; v + 1 < vhi; v += 2) {
        step(Rg[0], Rg[1], v, (v - vlo) & 1);
        step(Rg[1], Rg[0], v + 1, (v + 1 - vlo) & 1);
    }
    if (v < vhi) step(Rg[0], Rg[1], v, (v - vlo) & 1);
    if constexpr (NDOT > 0) reduce_finish<NDOT>(acc, R);
}

}  // namespace pp
