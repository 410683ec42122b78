// pp_march.hpp -- plane-marching stencil kernels (gfx950).
//
// The same operations as the per-cell kernels in pp_kernels.hpp, organised so
// that each array element is read from global memory about once per pass.  A
// block of 256 threads owns a BX x BY tile of cells (BX = 64, 32, 16 or 8) and
// walks a range of z planes.  The value the stencil needs at a neighbour (x,
// the red-cell value of a first sweep, the new search direction, ...) is
// formed once per cell: the z neighbours come from a three-plane register
// queue of the thread's own column, the in-plane neighbours from a
// double-buffered LDS copy of the current plane, and only threads on the tile
// edge read a halo value from global memory.  The west and south face weights
// of a cell are the east / north weights of its neighbours and come from LDS as
// well; the lower z face weight is carried over from the previous plane.
//
// One barrier per plane: a thread writes LDS buffer (k - k0) & 1, and a buffer
// is written again only two planes later, after every thread has passed the
// barrier that follows its last read of it.  The barrier waits for LDS only
// (not for the global loads in flight), and the global loads of plane
// k + kMarchSets - 1 are issued before the barrier of plane k into a rotating
// set of registers, so a wavefront keeps kMarchSets - 1 planes of loads
// outstanding while it works on the current one.
#pragma once
#include "pp_kernels.hpp"

namespace pp {

template <class T>
struct Stencil {
    T s;  // sum_f W_f v_nb(f)
    T d;  // sum_f W_f = D_c
    T ww, we, ws, wn, wb, wt;  // the face weights themselves (zero on walls)
};

struct None {};

// Tile of this block.  Blocks are dealt to the 8 XCDs round-robin (block b
// runs on XCD b mod 8), and each XCD has its own L2.  So that tiles sharing
// halo rows and columns share an L2, the b-th block takes tile
// (b mod 8) * (nblocks / 8) + b / 8 in x-fastest order: every XCD works on a
// contiguous run of tiles.  Launches whose block count is not a multiple of 8
// (or with xcd = 0) keep the plain order.
__device__ inline void tile_of_block(int& bx, int& by, int& bz, int xcd)
{
    const int gx = gridDim.x, gy = gridDim.y;
    const int nb = gx * gy * gridDim.z;
    const int b = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const int t = (!xcd || (nb & 7)) ? b : (b & 7) * (nb >> 3) + (b >> 3);
    bx = t % gx;
    by = (t / gx) % gy;
    bz = t / (gx * gy);
}

// LDS stores of this wavefront complete, then the work-group barrier.  Global
// loads still in flight are not waited for (each is waited for where its
// register is used).
__device__ inline void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// An operation supplies
//   Raw  load(c, i, j, k)  the global inputs of the stencil value at a cell,
//   T    val(raw)          the stencil value formed from them,
//   Ex   extra(c)          further per-cell inputs of apply,
//   void apply(c, i, j, k, v_c, raw_c, ex, st, acc, active)
// where st holds the stencil sums of val over the six neighbours of cell c.
// Every thread of the block calls apply at every plane (active is false
// outside the grid) so that apply may use wavefront shuffles.  val at a
// neighbour must not be changed by the pass itself (the callers write other
// arrays, or only cells of the colour that val is not read at).
// Threads of a march block: 256, or 512 for float64 on the finest level (tiles
// of 64 x 8: two halo rows for eight tile rows instead of for four; measured
// faster for the float64 kernels, slower for the float32 ones).
template <class T, bool RHO>
constexpr int kMarchThreads = (RHO && sizeof(T) == 8) ? 512 : kBlock;

// Where a march kernel's face weights come from (its WM parameter): the level's
// stored arrays in the kernel's precision, the density (finest level), or
// bfloat16 copies of the stored weights (coarse levels of the float32
// preconditioner: 6 bytes per cell instead of 12).
enum : int { kWStored = 0, kWRho = 1, kWHalf = 2 };

// Register sets of plane loads (loads are issued kMarchSets - 1 planes ahead
// of the plane being computed).
constexpr int kMarchSets = 2;

// Global inputs of one plane k of the tile: own face weights, apply's extras,
// the halo neighbour values (raw) and halo weights, and the raw inputs at k+1.
template <class T, class Raw, class Ex>
struct PlaneRegs {
    T wx, wy, wz, wxh, wyh;  // weights from memory; with the density: -, -, rho at k+1, halo rho x, halo rho y
    Raw rx, ry, rn;
    Ex ex;
};

// Face weight beta_f = 2 / (rho_L + rho_R) of the finest level (symmetric in
// L and R).  Float64: the IEEE division of the set-up, bit for bit; float32
// (preconditioner only): the hardware reciprocal.
__device__ inline double face_beta(double a, double b) { return 2.0 / (a + b); }
__device__ inline float face_beta(float a, float b) { return 2.0f * __builtin_amdgcn_rcpf(a + b); }

// Gauss-Seidel value (s + f) / D at a cell whose diagonal D is the sum of its
// face weights (the stencil's own d): no 1/D array is read.  Float64 divides;
// float32 (preconditioner only) multiplies by the hardware reciprocal.
__device__ inline double gs_value(double s, double f, double d) { return (s + f) / d; }
__device__ inline float gs_value(float s, float f, float d) { return (s + f) * __builtin_amdgcn_rcpf(d); }

// RHO: the level is the finest and its face weights are formed from L.rho
// (the x and y weights of a cell from the LDS copy of the plane's density,
// the z weight from the density of the next plane) instead of read from
// L.wx, L.wy, L.wz: 8 bytes per cell in float64 instead of 24.
//
// OVL (overlapped tiles, for operations that need values two cells away): the
// block's NT threads cover BX x BY cells of which the inner (BX-2) x (BY-2) are
// its own, tiles step by the inner size, the outer ring is computed again by
// the neighbouring blocks, and the march runs one plane below and one above
// the block's z range (periodic in z).  apply then sees ring cells and the two
// extra planes as well; cells outside the grid have act false.
template <class T, int BX, int WM, bool OVL = false, int NT = kMarchThreads<T, WM == kWRho>, class Op, class Acc>
__device__ inline void march(const LevelView<T>& L, int kper, int xcd, Op& op, Acc& acc)
{
    constexpr bool RHO = WM == kWRho, HALF = WM == kWHalf;
    using Raw = typename Op::Raw;
    using Ex = typename Op::Ex;
    using Regs = PlaneRegs<T, Raw, Ex>;
    constexpr int BY = NT / BX;
    constexpr int SX = OVL ? BX - 2 : BX, SY = OVL ? BY - 2 : BY, OFS = OVL ? 1 : 0;
    static_assert(BX >= 2 && BY >= 2, "a thread is on at most one x edge and one y edge of the tile");
    __shared__ T sv[2][BY][BX];
    __shared__ T swx[2][BY][BX];
    __shared__ T swy[2][BY][BX];
    const int tx = threadIdx.x, ty = threadIdx.y;
    int bx, by, bz;
    tile_of_block(bx, by, bz, xcd);
    const int i = bx * SX + tx - OFS, j = by * SY + ty - OFS;
    const int k0 = bz * kper, k1 = min(L.nz, k0 + kper);
    // planes marched, as virtual indices v (the plane is v mod nz with OVL)
    const int vlo = OVL ? k0 - 1 : k0, vhi = OVL ? k1 + 1 : k1;
    const bool act = i >= 0 && j >= 0 && i < L.nx && j < L.ny;
    const int sy = L.nx, sz = L.nx * L.ny;
    // Every load is issued by every lane at an address inside the grid (threads
    // outside it read the nearest cell, edge threads without a halo neighbour
    // read their own cell) and unused values are discarded: each plane issues
    // the same loads, so the compiler waits for exactly the ones it needs.
    const int ic = max(0, min(i, L.nx - 1)), jc = max(0, min(j, L.ny - 1));
    const int cbase = cell(L.nx, L.ny, ic, jc, 0);
    auto plane = [&](int v) { return OVL ? (v < 0 ? v + L.nz : (v >= L.nz ? v - L.nz : v)) : v; };
    const bool hx = act && ((tx == 0 && i > 0) || (tx == BX - 1 && i < L.nx - 1));
    const bool hy = act && ((ty == 0 && j > 0) || (ty == BY - 1 && j < L.ny - 1));
    const int oi = hx ? (tx == 0 ? -1 : 1) : 0;  // x offset of this thread's halo neighbour
    const int oj = hy ? (ty == 0 ? -1 : 1) : 0;
    const int owx = oi < 0 ? -1 : 0;             // the west face weight read from global memory
    const int owy = oj < 0 ? -sy : 0;
    const bool in_e = i < L.nx - 1, in_n = j < L.ny - 1;

    auto fetch = [&](Regs& S, int k, int c) {
        const int kt = k < L.nz - 1 ? k + 1 : 0;
        if constexpr (RHO) {
            // the cell's own density is the previous plane's z load (carried in rho_c)
            S.wx = T(0);
            S.wy = T(0);
            S.wz = L.rho[c + (kt - k) * sz];
            S.wxh = L.rho[c + oi];
            S.wyh = L.rho[c + oj * sy];
        } else if constexpr (HALF) {
            S.wx = (T)from_bf16(L.hwx[c]);
            S.wy = (T)from_bf16(L.hwy[c]);
            S.wz = (T)from_bf16(L.hwz[c]);
            S.wxh = (T)from_bf16(L.hwx[c + owx]);
            S.wyh = (T)from_bf16(L.hwy[c + owy]);
        } else {
            S.wx = L.wx[c];
            S.wy = L.wy[c];
            S.wz = L.wz[c];
            S.wxh = L.wx[c + owx];
            S.wyh = L.wy[c + owy];
        }
        S.ex = op.extra(c);
        S.rn = op.load(c + (kt - k) * sz, ic, jc, kt);
        S.rx = op.load(c + oi, ic + oi, jc, k);
        S.ry = op.load(c + oj * sy, ic, jc + oj, k);
    };

    // prologue: value at the plane below the first, value and raw inputs at the
    // first, registers of the first plane
    const int ks = plane(vlo), kb0 = ks > 0 ? ks - 1 : L.nz - 1;
    const int c = cbase + ks * sz;
    const T vm0 = op.val(op.load(c + (kb0 - ks) * sz, ic, jc, kb0));
    T wzb;
    T rho_c = T(0);  // RHO: density of the current plane's cell
    if constexpr (RHO) {
        rho_c = L.rho[c];
        wzb = face_beta(L.rho[c + (kb0 - ks) * sz], rho_c);
    } else if constexpr (HALF) {
        wzb = (T)from_bf16(L.hwz[c + (kb0 - ks) * sz]);
    } else {
        wzb = L.wz[c + (kb0 - ks) * sz];
    }
    Raw rc = op.load(c, ic, jc, ks);
    // kMarchSets register sets: plane v is in set (v - vlo) mod kMarchSets and the
    // loads of plane v + kMarchSets - 1 are issued while plane v is computed
    Regs R[kMarchSets];
#pragma unroll
    for (int s = 0; s < kMarchSets - 1; ++s) {
        const bool in = vlo + s < vhi;
        const int kf = in ? plane(vlo + s) : ks;
        fetch(R[s], kf, cbase + kf * sz);
    }
    T vm = act ? vm0 : T(0);
    T vc = act ? op.val(rc) : T(0);

    // One plane: S holds plane v, N receives plane v + kMarchSets - 1 (plane v
    // again near the block's last plane, unused).
    auto step = [&](Regs& S, Regs& N, int v, int buf) {
        constexpr int ahead = kMarchSets - 1;
        const int k = plane(v), c = cbase + k * sz;
        const bool more = v + ahead < vhi;
        const int kn = more ? plane(v + ahead) : k;
        fetch(N, kn, cbase + kn * sz);
        const T vp = act ? op.val(S.rn) : T(0);
        const T vxh = hx ? op.val(S.rx) : T(0);
        const T vyh = hy ? op.val(S.ry) : T(0);
        sv[buf][ty][tx] = vc;
        if constexpr (RHO) {
            swx[buf][ty][tx] = act ? rho_c : T(1);
        } else {
            swx[buf][ty][tx] = act ? S.wx : T(0);
            swy[buf][ty][tx] = act ? S.wy : T(0);
        }
        lds_barrier();
        const T vw = tx > 0 ? sv[buf][ty][tx - 1] : vxh;
        const T ve = tx < BX - 1 ? (in_e ? sv[buf][ty][tx + 1] : T(0)) : vxh;
        const T vs = ty > 0 ? sv[buf][ty - 1][tx] : vyh;
        const T vn = ty < BY - 1 ? (in_n ? sv[buf][ty + 1][tx] : T(0)) : vyh;
        T ww, we, ws, wn, wt;
        if constexpr (RHO) {
            // neighbour densities: LDS inside the tile, the halo value on its edge
            const T rc = rho_c;
            const T rw = tx > 0 ? swx[buf][ty][tx - 1] : S.wxh;
            const T re = tx < BX - 1 ? swx[buf][ty][tx + 1] : S.wxh;
            const T rs = ty > 0 ? swx[buf][ty - 1][tx] : S.wyh;
            const T rn = ty < BY - 1 ? swx[buf][ty + 1][tx] : S.wyh;
            ww = i > 0 ? face_beta(rw, rc) : T(0);
            we = in_e ? face_beta(rc, re) : T(0);
            ws = j > 0 ? face_beta(rs, rc) : T(0);
            wn = in_n ? face_beta(rc, rn) : T(0);
            wt = face_beta(rc, S.wz);
        } else {
            ww = i > 0 ? (tx > 0 ? swx[buf][ty][tx - 1] : S.wxh) : T(0);
            ws = j > 0 ? (ty > 0 ? swy[buf][ty - 1][tx] : S.wyh) : T(0);
            we = S.wx;
            wn = S.wy;
            wt = S.wz;
        }
        Stencil<T> st;
        st.s = ww * vw + we * ve + ws * vs + wn * vn + wzb * vm + wt * vp;
        st.d = ww + we + ws + wn + wzb + wt;
        st.ww = ww;
        st.we = we;
        st.ws = ws;
        st.wn = wn;
        st.wb = wzb;
        st.wt = wt;
        op.apply(c, i, j, k, vc, rc, S.ex, st, acc, act);
        vm = vc;
        vc = vp;
        rc = S.rn;
        wzb = wt;
        if constexpr (RHO) rho_c = S.wz;
    };

    // kMarchSets planes per trip so that the register sets rotate without copies
    int v = vlo;
    for (; v + kMarchSets - 1 < vhi; v += kMarchSets) {
#pragma unroll
        for (int s = 0; s < kMarchSets; ++s)
            step(R[s], R[(s + kMarchSets - 1) % kMarchSets], v + s, (v + s - vlo) & 1);
    }
#pragma unroll
    for (int s = 0; s < kMarchSets - 1; ++s)
        if (v + s < vhi) step(R[s], R[(s + kMarchSets - 1) % kMarchSets], v + s, (v + s - vlo) & 1);
}

// ---------------------------------------------------------------- operations

template <class T>
struct OpFirst {  // red-black SOR from a zero guess (red omega f/D, black one update)
    const T *f, *invd;
    T* x;
    T omega;
    struct Raw { T f, invd; };
    using Ex = None;
    __device__ Raw load(int c, int, int, int) const { return {f[c], invd[c]}; }
    __device__ T val(const Raw& a) const { return omega * (a.f * a.invd); }
    __device__ Ex extra(int) const { return {}; }
    template <class A>
    __device__ void apply(int c, int i, int j, int k, T vc, const Raw& a, const Ex&, const Stencil<T>& st, A&, bool act) const
    {
        if (!act) return;
        x[c] = (((i + j + k) & 1) == 0) ? vc : omega * ((st.s + a.f) * a.invd);
    }
};

// OpFirst on the K-cycle residual of the next step, f = r - alpha q (formed as
// the separate update forms it), which the pass also stores into fo (not r: the
// neighbouring blocks still read r).
template <class T>
struct OpFirstR {
    const T *r, *q, *invd;
    T* fo;
    T* x;
    T alpha, omega;
    struct Raw { T f, invd; };
    using Ex = None;
    __device__ Raw load(int c, int, int, int) const { return {r[c] - alpha * q[c], invd[c]}; }
    __device__ T val(const Raw& a) const { return omega * (a.f * a.invd); }
    __device__ Ex extra(int) const { return {}; }
    template <class A>
    __device__ void apply(int c, int i, int j, int k, T vc, const Raw& a, const Ex&, const Stencil<T>& st, A&, bool act) const
    {
        if (!act) return;
        fo[c] = a.f;
        x[c] = (((i + j + k) & 1) == 0) ? vc : omega * ((st.s + a.f) * a.invd);
    }
};

template <class T, int NDOT, class TQ>
struct OpHalf {  // one colour of a red-black SOR sweep in place; dots sum(x), <x, q>, <x, f>, sum(f) (NDOT 1-4)
    const T* f;
    T* x;
    const TQ* q;
    int colour;
    T omega;
    using Raw = T;
    struct Ex { T f; TQ q; };
    __device__ Raw load(int c, int, int, int) const { return x[c]; }
    __device__ T val(Raw a) const { return a; }
    __device__ Ex extra(int c) const { return {f[c], NDOT >= 2 ? q[c] : TQ(0)}; }
    template <class A>
    __device__ void apply(int c, int i, int j, int k, T vc, Raw, const Ex& e, const Stencil<T>& st, A& acc, bool act) const
    {
        if (!act) return;
        T xv = vc;
        if (((i + j + k) & 1) == colour) {
            xv = gs_value(st.s, e.f, st.d);
            if (omega != T(1)) xv = vc + omega * (xv - vc);
            x[c] = xv;
        }
        if constexpr (NDOT >= 1) acc[0] += (double)xv;
        if constexpr (NDOT >= 2) acc[1] += (double)xv * (double)e.q;
        if constexpr (NDOT >= 3) acc[2] += (double)xv * (double)e.f;
        if constexpr (NDOT >= 4) acc[3] += (double)e.f;
    }
};

template <class T>
struct OpProlongBlack {  // y = x + wc P e on red cells; black SOR update from them
    const T *f, *x, *e;
    T* y;
    T wc, omega;
    int cnx, cny;
    struct Raw { T x, e; };
    using Ex = T;  // f
    __device__ Raw load(int c, int i, int j, int k) const { return {x[c], e[cell(cnx, cny, i >> 1, j >> 1, k >> 1)]}; }
    __device__ T val(const Raw& a) const { return a.x + wc * a.e; }
    __device__ Ex extra(int c) const { return f[c]; }
    template <class A>
    __device__ void apply(int c, int i, int j, int k, T vc, const Raw&, const Ex& fc, const Stencil<T>& st, A&, bool act) const
    {
        if (!act) return;
        if (((i + j + k) & 1) == 0) {
            y[c] = vc;
        } else {
            T gs = gs_value(st.s, fc, st.d);
            if (omega != T(1)) gs = vc + omega * (gs - vc);
            y[c] = gs;
        }
    }
};

// d_new = (z - m) + b d_old (d_new = z - m without BETA), q = K d_new; dots
// <d,q> and <d,r> (FINE: <d,q> only; the finest level's step takes the
// numerator of its step length from the cycle's <z, r>, and r is not read).
// With BETA also the previous step's deferred update of x: XU 2 x += ap * d_old
// (the finest level's Krylov step, FINE), XU 1 x = ap * d_old (the second step
// of a K-cycle whose x starts at zero), XU 0 none.
template <class T, class TZ, bool BETA, bool FINE, int XU = FINE ? 2 : 0>
struct OpDir {
    static constexpr bool kDR = !FINE;  // the <d,r> dot
    const TZ* z;
    const T* dold;
    const T* r;
    T* dnew;
    T* q;
    T* x;
    T b, m, ap;
    struct Raw { TZ z; T d; };
    struct Ex { T r, x; };
    __device__ Raw load(int c, int, int, int) const { return {z[c], BETA ? dold[c] : T(0)}; }
    __device__ T val(const Raw& a) const { return BETA ? ((T)a.z - m) + b * a.d : ((T)a.z - m); }
    __device__ Ex extra(int c) const { return {kDR ? r[c] : T(0), (XU == 2 && BETA) ? x[c] : T(0)}; }
    template <class A>
    __device__ void apply(int c, int, int, int, T vc, const Raw& own, const Ex& ev, const Stencil<T>& st, A& acc,
                          bool act) const
    {
        if (!act) return;
        const T qc = st.d * vc - st.s;
        dnew[c] = vc;
        q[c] = qc;
        acc[0] += (double)vc * (double)qc;
        if constexpr (kDR) acc[1] += (double)vc * (double)ev.r;
        if constexpr (XU == 2 && BETA) x[c] = ev.x + ap * own.d;
        if constexpr (XU == 1 && BETA) x[c] = ap * own.d;
    }
};

template <class T>
struct OpResidual {  // r = f - K x; sums ||r||^2, sum r, sum x; optionally a copy of x and a float32 copy of r
    const T* f;
    const T* x;
    T* r;
    T* xc = nullptr;       // receives x (or null)
    float* r32 = nullptr;  // receives (float) r (or null)
    using Raw = T;
    using Ex = T;
    __device__ Raw load(int c, int, int, int) const { return x[c]; }
    __device__ T val(Raw a) const { return a; }
    __device__ Ex extra(int c) const { return f[c]; }
    template <class A>
    __device__ void apply(int c, int, int, int, T vc, Raw, Ex fc, const Stencil<T>& st, A& acc, bool act) const
    {
        if (!act) return;
        const T rv = fc - (st.d * vc - st.s);
        r[c] = rv;
        if (xc) xc[c] = vc;
        if (r32) r32[c] = (float)rv;
        acc[0] += (double)rv * (double)rv;
        acc[1] += (double)rv;
        acc[2] += (double)vc;
    }
};

template <class T>
struct OpApply {  // y = A x = -(K x) / h^2, the operator of step 11 on its own
    const T* x;
    T* y;
    T inv_h2;
    using Raw = T;
    using Ex = None;
    __device__ Raw load(int c, int, int, int) const { return x[c]; }
    __device__ T val(Raw a) const { return a; }
    __device__ Ex extra(int) const { return {}; }
    template <class A>
    __device__ void apply(int c, int, int, int, T vc, Raw, const Ex&, const Stencil<T>& st, A&, bool act) const
    {
        if (act) y[c] = (st.s - st.d * vc) * inv_h2;
    }
};

// ||bbar - A p||^2 and ||bbar||^2 with bbar = b - mean(b), the mean read from
// a slot: the relative residual of step 11 measured on the device.
struct OpRelResidual {
    const double* p;
    const double* b;
    double inv_h2, mean;
    using Raw = double;
    using Ex = double;
    __device__ Raw load(int c, int, int, int) const { return p[c]; }
    __device__ double val(Raw a) const { return a; }
    __device__ Ex extra(int c) const { return b[c]; }
    template <class A>
    __device__ void apply(int, int, int, int, double vc, Raw, Ex bc, const Stencil<double>& st, A& acc, bool act) const
    {
        if (!act) return;
        const double bb = bc - mean;
        const double r = bb - (st.s - st.d * vc) * inv_h2;
        acc[0] += r * r;
        acc[1] += bb * bb;
    }
};

// Residual f - K x summed over the 8 children of each coarse cell.  The 2 x 2
// children of a plane sit on lanes (l, l+1) of rows (ty, ty+1), which share a
// wavefront for BX <= 32; the two planes of a pair are consecutive steps of the
// march (the block's first plane and kper are even).
template <class T, int BX>
struct OpRestrict {
    const T* f;
    const T* x;
    T* rc;
    int cnx, cny, k0;
    T part;
    using Raw = T;
    using Ex = T;
    __device__ Raw load(int c, int, int, int) const { return x[c]; }
    __device__ T val(Raw a) const { return a; }
    __device__ Ex extra(int c) const { return f[c]; }
    template <class A>
    __device__ void apply(int c, int i, int j, int k, T vc, Raw, Ex fc, const Stencil<T>& st, A&, bool act)
    {
        const T rv = act ? fc - (st.d * vc - st.s) : T(0);
        T p = rv + __shfl_down(rv, 1, 64);
        p = p + __shfl_down(p, BX, 64);
        if (((k - k0) & 1) == 0) part = p;
        else if (act && ((threadIdx.x | threadIdx.y) & 1) == 0) rc[cell(cnx, cny, i >> 1, j >> 1, k >> 1)] = part + p;
    }
};

// Overlapped tile of m_first_restrict: 32 x 16 threads, 30 x 14 cells of its own.
constexpr int kOvlX = 32, kOvlY = 16;

// The first sweep from a zero guess (as OpFirst) and the restriction of its
// residual (as OpRestrict) in one pass.  A red cell's residual needs its black
// neighbours' new values, and those need their red neighbours, so the block
// computes x on its ring and on the planes below and above its range as well
// (march with OVL), writes x for its own cells and real planes only, and forms
// the residual one plane behind the sweep from the x values of three planes:
// the in-plane neighbours from an LDS copy of the previous plane, the z
// neighbours from registers.  The 2 x 2 children of a plane are lanes
// (l, l+1) of one row (one wavefront) and rows (t, t+1) summed through LDS;
// the two planes of a pair are consecutive steps (k0 and kper even).
template <class T>
struct OpFirstRestrict {
    const T *f, *invd;
    T* x;
    T* rc;
    T omega;
    int cnx, cny, k0, nreal;  // coarse sizes, first plane and real planes of the block
    int s = 0;                // step: plane k0 - 1 + s
    T xm2 = T(0), xm1 = T(0), fm1 = T(0), part = T(0);  // x two and one planes back, f one back
    T pw = T(0), pe = T(0), ps = T(0), pn = T(0), pb = T(0), pt = T(0);  // face weights one back
    struct Raw { T f, invd; };
    using Ex = None;
    __device__ Raw load(int c, int, int, int) const { return {f[c], invd[c]}; }
    __device__ T val(const Raw& a) const { return omega * (a.f * a.invd); }
    __device__ Ex extra(int) const { return {}; }
    template <class A>
    __device__ void apply(int c, int i, int j, int k, T vc, const Raw& a, const Ex&, const Stencil<T>& st, A&, bool act)
    {
        __shared__ T sx[2][kOvlY][kOvlX];  // x of the last two planes
        __shared__ T sr[kOvlY][kOvlX];     // restriction sums of the rows
        const int tx = threadIdx.x, ty = threadIdx.y;
        const T xv = act ? ((((i + j + k) & 1) == 0) ? vc : omega * ((st.s + a.f) * a.invd)) : T(0);
        const bool own = act && tx >= 1 && tx <= kOvlX - 2 && ty >= 1 && ty <= kOvlY - 2;
        if (own && s >= 1 && s <= nreal) x[c] = xv;
        sx[s & 1][ty][tx] = xv;  // read at the next step, after its barrier
        if (s >= 2) {
            // residual of plane k0 - 2 + s (a real plane), from x of three planes
            T r = T(0);
            if (own) {
                const int b = (s - 1) & 1;
                const T nb = pw * sx[b][ty][tx - 1] + pe * sx[b][ty][tx + 1] + ps * sx[b][ty - 1][tx] +
                             pn * sx[b][ty + 1][tx] + pb * xm2 + pt * xv;
                const T d = pw + pe + ps + pn + pb + pt;
                r = fm1 - (d * xm1 - nb);
            }
            const T p = r + __shfl_down(r, 1, 64);  // x pairs: lanes (l, l+1) of one 32-lane row
            if ((s & 1) == 0) {
                part = p;  // even plane of the pair
            } else {
                const T p2 = part + p;
                sr[ty][tx] = p2;
                lds_barrier();
                if (own && (tx & 1) && (ty & 1))
                    rc[cell(cnx, cny, i >> 1, j >> 1, (k0 - 2 + s) >> 1)] = p2 + sr[ty + 1][tx];
            }
        }
        xm2 = xm1;
        xm1 = xv;
        fm1 = a.f;
        pw = st.ww;
        pe = st.we;
        ps = st.ws;
        pn = st.wn;
        pb = st.wb;
        pt = st.wt;
        ++s;
    }
};

// Prolongation with the black update (as OpProlongBlack) and the red half-sweep
// after it (as OpHalf with colour 0) in one pass, for a level smoothed once
// after the coarse correction.  The red update needs the new black values around
// it and those need the prolongated red values around them, so the march runs
// with overlapped tiles (OVL) and the red update trails the black one by a plane,
// as in OpFirstRestrict.  Writes z = y on black cells and the updated red cells;
// dots sum(z), <z, q>, <z, f> and sum(f) (NDOT 1-4) over the block's own cells.
template <class T, int NDOT, class TQ>
struct OpProlongHalf {
    const T *f, *x, *e;
    const TQ* q;
    T* z;
    T wc, omega;
    int cnx, cny;
    int s = 0;  // step: plane k0 - 1 + s
    T ym2 = T(0), ym1 = T(0), fm1 = T(0);  // y two and one planes back, f one back
    TQ qm1 = TQ(0);
    int cm1 = 0, km1 = 0;                  // cell index and plane one back
    T pw = T(0), pe = T(0), ps = T(0), pn = T(0), pb = T(0), pt = T(0);
    struct Raw { T x, e; };
    struct Ex { T f; TQ q; };
    __device__ Raw load(int c, int i, int j, int k) const { return {x[c], e[cell(cnx, cny, i >> 1, j >> 1, k >> 1)]}; }
    __device__ T val(const Raw& a) const { return a.x + wc * a.e; }
    __device__ Ex extra(int c) const { return {f[c], NDOT >= 2 ? q[c] : TQ(0)}; }
    template <class A>
    __device__ void apply(int c, int i, int j, int k, T vc, const Raw&, const Ex& ex, const Stencil<T>& st, A& acc, bool act)
    {
        __shared__ T sy[2][kOvlY][kOvlX];  // y of the last two planes
        const int tx = threadIdx.x, ty = threadIdx.y;
        T yv = T(0);
        if (act) {
            if (((i + j + k) & 1) == 0) {
                yv = vc;
            } else {
                yv = gs_value(st.s, ex.f, st.d);
                if (omega != T(1)) yv = vc + omega * (yv - vc);
            }
        }
        const bool own = act && tx >= 1 && tx <= kOvlX - 2 && ty >= 1 && ty <= kOvlY - 2;
        sy[s & 1][ty][tx] = yv;  // read at the next step, after its barrier
        if (s >= 2 && own) {
            // plane km1 (a real plane of the block): red cells relaxed from y of three planes
            T zv = ym1;
            if (((i + j + km1) & 1) == 0) {
                const int b = (s - 1) & 1;
                const T nb = pw * sy[b][ty][tx - 1] + pe * sy[b][ty][tx + 1] + ps * sy[b][ty - 1][tx] +
                             pn * sy[b][ty + 1][tx] + pb * ym2 + pt * yv;
                zv = gs_value(nb, fm1, pw + pe + ps + pn + pb + pt);
                if (omega != T(1)) zv = ym1 + omega * (zv - ym1);
            }
            z[cm1] = zv;
            if constexpr (NDOT >= 1) acc[0] += (double)zv;
            if constexpr (NDOT >= 2) acc[1] += (double)zv * (double)qm1;
            if constexpr (NDOT >= 3) acc[2] += (double)zv * (double)fm1;
            if constexpr (NDOT >= 4) acc[3] += (double)fm1;
        }
        ym2 = ym1;
        ym1 = yv;
        fm1 = ex.f;
        qm1 = ex.q;
        cm1 = c;
        km1 = k;
        pw = st.ww;
        pe = st.we;
        ps = st.ws;
        pn = st.wn;
        pb = st.wb;
        pt = st.wt;
        ++s;
    }
};

// ---------------------------------------------------------------- kernels

template <class T, int BX, int WM>
__global__ void __launch_bounds__((kMarchThreads<T, WM == kWRho>)) m_smooth_first(LevelView<T> L, const T* __restrict__ f, T* __restrict__ x, int kper,
                                                        int xcd, T omega)
{
    OpFirst<T> op{f, L.invd, x, omega};
    double acc[1] = {0.0};
    march<T, BX, WM>(L, kper, xcd, op, acc);
}

template <class T, int BX, int WM, int NDOT, class TQ>
__global__ void __launch_bounds__((kMarchThreads<T, WM == kWRho>)) m_smooth_half(LevelView<T> L, const T* __restrict__ f, T* x, int colour, int kper,
                                                       int xcd, const TQ* __restrict__ q, Reduce R, T omega)
{
    OpHalf<T, NDOT, TQ> op{f, x, q, colour, omega};
    double acc[NDOT > 0 ? NDOT : 1] = {};
    march<T, BX, WM>(L, kper, xcd, op, acc);
    if constexpr (NDOT > 0) reduce_finish<NDOT>(acc, R);
}

template <class T, int BX, int WM>
__global__ void __launch_bounds__((kMarchThreads<T, WM == kWRho>)) m_residual_restrict(LevelView<T> L, const T* __restrict__ f, const T* __restrict__ x,
                                                             T* __restrict__ rc, int kper, int xcd)
{
    static_assert(BX <= 32, "the 2x2 sum pairs rows within one wavefront");
    int bx, by, bz;
    tile_of_block(bx, by, bz, xcd);
    OpRestrict<T, BX> op{f, x, rc, L.nx >> 1, L.ny >> 1, bz * kper, T(0)};
    double acc[1] = {0.0};
    march<T, BX, WM>(L, kper, xcd, op, acc);
}

template <class T, int WM>
__global__ void __launch_bounds__(kOvlX * kOvlY) m_first_restrict(LevelView<T> L, const T* __restrict__ f, T* __restrict__ x,
                                                                 T* __restrict__ rc, int kper, int xcd, T omega)
{
    int bx, by, bz;
    tile_of_block(bx, by, bz, xcd);
    const int k0 = bz * kper;
    OpFirstRestrict<T> op{f, L.invd, x, rc, omega, L.nx >> 1, L.ny >> 1, k0, min(L.nz, k0 + kper) - k0};
    double acc[1] = {0.0};
    march<T, kOvlX, WM, true, kOvlX * kOvlY>(L, kper, xcd, op, acc);
}

template <class T, int WM, int NDOT, class TQ>
__global__ void __launch_bounds__(kOvlX * kOvlY) m_prolong_half(LevelView<T> L, const T* __restrict__ f,
                                                               const T* __restrict__ x, const T* __restrict__ e, T wc,
                                                               T* __restrict__ z, const TQ* __restrict__ q, Reduce R,
                                                               int kper, int xcd, T omega)
{
    OpProlongHalf<T, NDOT, TQ> op{f, x, e, q, z, wc, omega, L.nx >> 1, L.ny >> 1};
    double acc[NDOT > 0 ? NDOT : 1] = {};
    march<T, kOvlX, WM, true, kOvlX * kOvlY>(L, kper, xcd, op, acc);
    if constexpr (NDOT > 0) reduce_finish<NDOT>(acc, R);
}

template <class T, int BX, int WM>
__global__ void __launch_bounds__((kMarchThreads<T, WM == kWRho>)) m_prolong_black(LevelView<T> L, const T* __restrict__ f, const T* __restrict__ x,
                                                         const T* __restrict__ e, T wc, T* __restrict__ y, int kper, int xcd,
                                                         T omega)
{
    OpProlongBlack<T> op{f, x, e, y, wc, omega, L.nx >> 1, L.ny >> 1};
    double acc[1] = {0.0};
    march<T, BX, WM>(L, kper, xcd, op, acc);
}

template <class T, int BX, int WM, class TZ, bool BETA, bool FINE>
__global__ void __launch_bounds__((kMarchThreads<T, WM == kWRho>)) m_dir_apply(LevelView<T> L, const TZ* __restrict__ z, const T* __restrict__ dold,
                                                     T* __restrict__ dnew, T* __restrict__ q, const T* __restrict__ r,
                                                     T* __restrict__ x, Coefs beta, Coefs mean, int use_mean, Coefs aprev,
                                                     int kper, int xcd, Reduce R)
{
    OpDir<T, TZ, BETA, FINE> op{z, dold, r, dnew, q, x, BETA ? (T)beta.get() : T(0), use_mean ? (T)mean.get() : T(0),
                                (FINE && BETA) ? (T)aprev.get() : T(0)};
    constexpr int NV = FINE ? 1 : 2;
    double acc[NV] = {};
    march<T, BX, WM>(L, kper, xcd, op, acc);
    reduce_finish<NV>(acc, R);
}

// y = A x on the finest level with the march kernels' weights (the same tiles,
// neighbour exchange and density-formed face coefficients as the solve's passes).
template <int BX, int WM>
__global__ void __launch_bounds__((kMarchThreads<double, WM == kWRho>)) m_apply(LevelView<double> L, const double* __restrict__ x,
                                                                             double* __restrict__ y, double inv_h2,
                                                                             int kper, int xcd)
{
    OpApply<double> op{x, y, inv_h2};
    double acc[1] = {0.0};
    march<double, BX, WM>(L, kper, xcd, op, acc);
}

// Sums of OpRelResidual over the grid (weights formed from the density).
template <int BX>
__global__ void __launch_bounds__((kMarchThreads<double, true>)) m_rel_residual(LevelView<double> L, const double* __restrict__ p,
                                                                              const double* __restrict__ b, double inv_h2,
                                                                              Coefs mean, int kper, Reduce R)
{
    OpRelResidual op{p, b, inv_h2, mean.get()};
    double acc[2] = {0.0, 0.0};
    march<double, BX, kWRho>(L, kper, 0, op, acc);
    reduce_finish<2>(acc, R);
}

template <int BX, int WM>
__global__ void __launch_bounds__((kMarchThreads<double, WM == kWRho>)) m_true_residual(LevelView<double> L, const double* __restrict__ f,
                                                         const double* __restrict__ x, double* __restrict__ r, int kper, int xcd,
                                                         Reduce R, double* __restrict__ xc, float* __restrict__ r32)
{
    OpResidual<double> op{f, x, r, xc, r32};
    double acc[3] = {0.0, 0.0, 0.0};
    march<double, BX, WM>(L, kper, xcd, op, acc);
    reduce_finish<3>(acc, R);
}

}  // namespace pp
