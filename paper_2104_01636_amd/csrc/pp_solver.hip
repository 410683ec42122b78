// pp_solver.hip -- host side of the pressure solver: hierarchy, Krylov drivers, C ABI.
//
// Method.  The paper solves its pressure equations on the GPU by red-black SOR
// relaxation, accelerated by multigrid (Section 2.1, after eq.
// ppe_surface_tension), and gives no further detail.  Here the same pieces
// -- red-black Gauss-Seidel relaxation and geometric multigrid -- precondition
// a conjugate-gradient iteration:
//   * finest level: flexible CG (one-term recurrence) on K p = f;
//   * preconditioner: one multigrid cycle with red-black Gauss-Seidel
//     (red then black before the coarse correction, black then red after),
//     residual restriction by summing the 8 children, injection prolongation
//     and Galerkin coarse operators (face sums);
//   * coarse levels 1..kmax are "K-cycles": the coarse problem is solved by a
//     few flexible-CG steps preconditioned by the next cycle; deeper levels use
//     a plain V-cycle whose correction is scaled by wc; the coarsest level is
//     solved with a dense inverse of K + (mean D / n) 1 1^T.
// The preconditioner only changes the iteration count; the converged result is
// the zero-mean solution of A p = b - mean(b).
//
// Mixed precision: in PP_FP32_REFINED mode the outer flexible CG stays
// float64 (x, r, d, q and the operator built from rho), and only the
// multigrid preconditioner runs in float32 on a float32 copy of r (dot
// products accumulate in float64).  A preconditioner only has to be a fair
// approximation of K^-1, so its rounding changes the iteration count, not the
// accuracy reached; an iterative refinement with a float32 inner Krylov solve
// instead stalls once kappa(K) * 2^-24 approaches one (kappa is about 1e7 for
// a 128^2 x 256 grid with a 1000:1.2 density ratio).
//
// Stencil passes on levels with more cells than the single-workgroup tail use
// the plane-marching kernels of pp_march.hpp (PP_MARCH=0 selects the simpler
// one-thread-per-column kernels of pp_kernels.hpp, kept as a reference form).
#include "pp_kernels.hpp"
#include "pp_march.hpp"
#include "pp_tail.hpp"
#include "pp_rowwave.hpp"
#include "pp_rowfused.hpp"
#include "../../include/pp.h"

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

namespace pp {

static thread_local std::string g_thread_err = "no error";

#define PP_HIP(expr)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) {                                                                        \
            throw Fail(PP_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));                 \
        }                                                                                              \
    } while (0)

struct Fail {
    int code;
    std::string msg;
    Fail(int c, std::string m) : code(c), msg(std::move(m)) {}
};

// ---------------------------------------------------------------- launch geometry

struct Geo {
    dim3 grid, block;
    int kper;
};

static Geo geo(int nx, int ny, int nz, int max_blocks = kMaxRedBlocks)
{
    int bx = 1;
    while (bx < nx && bx < 64) bx <<= 1;
    int by = kBlock / bx;
    while (by > 1 && by / 2 >= ny) by >>= 1;
    int gx = (nx + bx - 1) / bx, gy = (ny + by - 1) / by;
    int tiles = gx * gy;
    int gz = std::max(1, std::min(nz, max_blocks / std::max(1, tiles)));
    int kper = (nz + gz - 1) / gz;
    gz = (nz + kper - 1) / kper;
    return {dim3(gx, gy, gz), dim3(bx, by, 1), kper};
}

// Plane-march geometry: tiles of bx x (256 / bx) cells, bx a power of two in
// [8, bx_max] not far above nx; z split so that the launch has at most
// kMaxRedBlocks blocks; kper even when the kernel pairs planes.
struct MGeo {
    dim3 grid, block;
    int kper, bx;
};

static MGeo mgeo(int nx, int ny, int nz, int bx_max, bool even_k = false, int max_blocks = kMaxRedBlocks,
                 int threads = kBlock)
{
    int bx = 8;
    while (bx < nx && bx < bx_max) bx <<= 1;
    const int by = threads / bx;
    const int gx = (nx + bx - 1) / bx, gy = (ny + by - 1) / by;
    const int tiles = gx * gy;
    int gz = std::max(1, std::min(nz, max_blocks / std::max(1, tiles)));
    int kper = (nz + gz - 1) / gz;
    if (even_k && (kper & 1)) ++kper;
    gz = (nz + kper - 1) / kper;
    return {dim3(gx, gy, gz), dim3(bx, by, 1), kper, bx};
}

// Geometry of an overlapped-tile launch (m_first_restrict): tiles of
// (kOvlX - 2) x (kOvlY - 2) own cells, z split into an even number of planes
// per block so that plane pairs stay in one block.  nz is even.
static MGeo ovl_geo(int nx, int ny, int nz, int max_blocks)
{
    const int gx = (nx + kOvlX - 3) / (kOvlX - 2), gy = (ny + kOvlY - 3) / (kOvlY - 2);
    const int tiles = gx * gy;
    int gz = std::max(1, std::min(nz / 2, max_blocks / std::max(1, tiles)));
    int kper = (nz + gz - 1) / gz;
    if (kper & 1) ++kper;
    gz = (nz + kper - 1) / kper;
    return {dim3(gx, gy, gz), dim3(kOvlX, kOvlY, 1), kper, kOvlX};
}

template <int B>
using BxC = std::integral_constant<int, B>;

// Calls f(BxC<bx>{}) for the tile widths the march kernels are built for.
template <class F>
static void with_bx(int bx, F&& f)
{
    switch (bx) {
    case 8: f(BxC<8>{}); break;
    case 16: f(BxC<16>{}); break;
    case 32: f(BxC<32>{}); break;
    default: f(BxC<64>{}); break;
    }
}
template <class F>
static void with_bx_le32(int bx, F&& f)
{
    switch (bx) {
    case 8: f(BxC<8>{}); break;
    case 16: f(BxC<16>{}); break;
    default: f(BxC<32>{}); break;
    }
}

static dim3 lin_grid(size_t n)
{
    size_t b = (n + kBlock - 1) / kBlock;
    return dim3((unsigned)std::max<size_t>(1, std::min<size_t>(b, kMaxRedBlocks)));
}

// ---------------------------------------------------------------- slots

enum : int {
    kLevSlots = 8,      // per level: ZQ, SUMZ, DQ0, DQ1, DR, RR, RSUM
    S_ZQ = 0, S_SUMZ = 1, S_DQ0 = 2, S_DQ1 = 3, S_DR = 4, S_RR = 5, S_RSUM = 6,
    G_BASE = 200,
    G_BSUM = G_BASE + 0, G_BBAD = G_BASE + 1, G_FN2 = G_BASE + 2, G_TRR = G_BASE + 3, G_TRSUM = G_BASE + 4,
    G_XSUM = G_BASE + 5, G_XBAD = G_BASE + 6, G_SCALE = G_BASE + 7, G_INVSCALE = G_BASE + 8, G_RHOSUM = G_BASE + 9,
    G_RHOBAD = G_BASE + 10, G_ONE = G_BASE + 11, G_ZERO = G_BASE + 12,
    G_ALPHA0 = G_BASE + 13, G_ALPHA1 = G_BASE + 14,  // the finest level's step lengths, by step parity
    G_FSUM = G_BASE + 15,                            // sum of the residual the finest cycle read
    kSlots = 256
};
static inline int lslot(int l, int s) { return l * kLevSlots + s; }

constexpr int kMaxLev = 24;
constexpr int kDenseMax = kDenseRows;  // coarsening stops at the first level of at most this many cells
static_assert(kDenseMax <= kTailDenseMax, "the tail's dense product covers the coarsest level");

// ---------------------------------------------------------------- arena plan

struct Level64 {  // float64 coefficients of a coarse level (set-up and float64 mode)
    double *wx = nullptr, *wy = nullptr, *wz = nullptr, *invd = nullptr;
};
struct Level32 {
    float *wx = nullptr, *wy = nullptr, *wz = nullptr, *invd = nullptr;
    unsigned short *hx = nullptr, *hy = nullptr, *hz = nullptr;  // bfloat16 weights (coarse levels)
};

template <class T>
struct Lev {
    int nx, ny, nz;
    size_t n;
    LevelView<T> v;
    bool kcyc;            // solved by K-cycle steps
    T *rhs = nullptr, *c = nullptr, *c2 = nullptr;
    T *xk = nullptr, *d = nullptr, *d2 = nullptr, *q = nullptr;  // Krylov levels
    T* rhs2 = nullptr;                 // K-cycle: the other residual buffer (float32 levels)
    T *d_a = nullptr, *d_b = nullptr;  // the two search-direction buffers (d, d2 alternate between them)
    T *w1 = nullptr, *rr = nullptr;    // W-cycle: the first visit's correction, the coarse residual
};

// Event pair around one timed launch (see TimeScope).
struct TimedPair {
    int id;
    double bytes;
    hipEvent_t a, b;
};

// Multigrid hierarchy in the preconditioner's precision T.  Level 0 holds only
// the cycle's input (rhs) and output buffers; the finest-level Krylov vectors
// are float64 and live in the Handle.
template <class T>
struct Hier {
    std::vector<Lev<T>> L;
    T* Minv = nullptr;   // coarsest dense inverse (when n <= kDenseMax)
    int nd = 0;
    int tail = -1;       // first level of the single-launch tail V-cycle (-1: none)
    TailDesc<T> td{};
};

struct Params {
    int nu0 = 1, nuc = 2, kmax = 2, kit = 3, coarse_sweeps = 16;
    int kit2 = 4;               // K-cycle steps on the deepest K-cycle level (the one whose coarse
                                // correction is a plain V-cycle) when it has more than kbig cells
    long kbig = 262144;         // (measured: 4 steps faster on 524288-cell levels, 3 on 221184)
    int nuk2 = 1;               // sweeps on the K-cycle levels >= 2 (0: nuc); the extra
                                // K-cycle step there buys more than the second sweep
    int nuv = 1;                // sweeps on the V-cycle levels below the K-cycles (0: nuc)
    int nu1 = 0;                // sweeps on level 1 (0: nuc)
    bool tail = true;           // run the small coarse V-levels in one launch
    int kmin = 65536;           // K-cycles only on levels with more cells than this (smaller ones: V-cycles,
                                // whose launches cost less than the iterations they save)
    int tail_max = 1024;        // largest level the one-launch cycle starts on (at most kTailMaxCells)
    double wc = 2.0;
    bool graphs = true;
    bool hw = true;             // bfloat16 face weights for the float32 cycle below the finest level,
    long hwmin = 65536;         // on levels with more cells than this (the bandwidth-bound ones; on
                                // small grids the 8-bit significand costs iterations)
    int fuse = 1;               // levels smoothed once: first sweep with restriction, and
                                // prolongation with the last half-sweep, as overlapped-tile
                                // launches on float32 levels (1), on every level (2) or nowhere
                                // (0); measured faster in float32 only (the float64 launches
                                // hold fewer waves per CU)
    int oblocks = 3072;         // block budget of an overlapped-tile launch
    int pfuse = 1;              // fuse the post-smoothing too (the pre-smoothing always when fused)
    long fbig = 1L << 20;       // fused launches on levels with at least fbig cells (the ring and the
    long fsmall = 65536;        // two extra planes cost little) or at most fsmall (bound by launch
                                // latency); between them the overlap costs more than it saves
    double omega = 1.0;         // SOR factor of the red-black smoother
    bool mg_solver = false;     // multigrid cycles as the solver (no Krylov outer iteration)
    int gamma = 1;              // coarse-grid visits per cycle in that form: 1 V-cycle, 2 W-cycle
    bool march = true;          // plane-marching stencil kernels (else one thread per cell column)
    int mbx = 64;               // widest march tile in x
    int mblocks = 768;          // blocks of a 256-thread march launch (at most; z split to reach it)
    int fblocks = 512;          // blocks of a 512-thread (finest-level float64) march launch
    int xcd = 2;                // XCD-aware tile order: 0 never, 1 always, 2 below the finest level
    int oxcd = 1;               // the same for the overlapped-tile launches (-1: as xcd); their
                                // ring rows then come from the L2 of the XCD, measured 3 % faster
    bool rho = true;            // finest-level march kernels form the weights from the density
    bool rw = true;             // row-wave kernels (whole rows) for the finest-level float64 residual and
                                // operator when nx is 64, 128, 192 or 256
    int rwsplit = 2;            // wavefronts per row of those passes where nx is 128 or 256: 1 or 2 (a
                                // row over two wavefronts holds half the cells per lane: 3-4 waves
                                // per SIMD instead of 2 for the direction update)
    int rwdir = 2;              // row-wave direction update: 0 never, 1 always, 2 with split rows (one
                                // wavefront per row measured slower than the tiles: 415 against 402 us;
                                // split rows faster: 366 us)
    int rwblocks = 512;         // blocks of a finest-level row-wave launch, at most (z split to reach it),
    int rwrows = 8;             // rows per block (4 or 8) and band order, one wavefront per row
    int rwsblocks = 256;        // the same with split rows (rows 4, 6 or 8), measured best at 256 blocks
    int rwsrows = 4;            // of 4 rows in the XCD band order (the direction update 312 us; plain
    int rwsxcd = 1;             // order 317, 8 rows 327-332, 6 rows 351, 512 blocks 321)
    int eblocks = 512;          // blocks of the finest-level r/q update, at most (164 us with 512, 185
                                // with 2048, 215 with 256)
    bool onepass = true;        // the finest level's set-up and the first coarse level's weights in one
                                // pass over the density (k_fine_setup; the same values as the separate
                                // passes)
    bool kfold = true;          // K-cycle steps on row-wave float32 levels without a separate x/r update:
                                // r -= alpha q rides on the next step's first sweep, x += alpha d on
                                // the next step's direction update
    int rwcrows = 8;            // rows of a coarse-level row-wave block: 4 or 8
    int rwcblocks = 512;        // blocks of a coarse-level row-wave launch, at most
    int rwcxcd = 1;             // XCD-aware band order for them
    bool rwc = true;            // row-wave passes on float32 coarse levels with bfloat16 weights (nx 64..256)
    bool rwf = true;            // row-wave forms of the fused float32 finest-level passes (nx 128 or 256)
    int rwfrows = 12;           // their rows per block, ring included: 8, 12 or 16 (12: the most rows whose
                                // registers (153 per lane) still fit three waves per SIMD)
    int rwfblocks = 256;        // their blocks per launch, at most (one per CU)
    int rwfxcd = 0;             // XCD-aware band order for them (measured slower: 265 against 213 us)
    int rwxcd = 1;              // XCD-aware band order for the finest-level row-wave launches with one
                                // wavefront per row (neighbouring row bands, whose halo rows overlap,
                                // share an L2)
};

struct Handle {
    pp_config cfg{};
    hipStream_t user = nullptr;    // caller's stream (may be the null stream)
    hipStream_t stream = nullptr;  // the handle's own stream; ordered after / before `user` by events
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    int device = 0;
    Params prm;
    std::string err = "no error";
    bool have_density = false;
    int zr_slot = 0;               // slots of <z, f> and sum(f) for a cycle's third and fourth dots (ndot 4)
    int fsum_slot = 0;

    // geometry of levels
    std::vector<int> lnx, lny, lnz;
    int nlev = 0;

    // arena
    char* arena = nullptr;
    size_t arena_bytes = 0;

    // face weights per level (c64[0] holds beta_f of the finest level)
    std::vector<Level64> c64;
    std::vector<Level32> c32;
    double* M64 = nullptr;
    float* M32 = nullptr;

    // float64 finest-level Krylov state (both modes): scaled right-hand side f,
    // residual r, iterate x, search directions (d, d2 alternate between d_a and
    // d_b), q = K d; r32 = float32 copy of r for a float32 preconditioner
    double *f64 = nullptr, *r64 = nullptr, *x64 = nullptr, *q64 = nullptr;
    double *d = nullptr, *d2 = nullptr, *d_a = nullptr, *d_b = nullptr;
    float* r32 = nullptr;
    double* rho64 = nullptr;   // copy of the density (finest-level weights of the plane-marching kernels)
    float* rho32 = nullptr;    // its float32 copy (float32 preconditioner)
    // captured Krylov steps: [0] first step, [1] odd steps, [2] even steps >= 2
    hipGraphExec_t kexec[3] = {nullptr, nullptr, nullptr};

    Hier<double> h64;
    Hier<float> h32;

    // reductions
    double* partials = nullptr;
    double* slots = nullptr;
    double* host_slots = nullptr;  // pinned, mapped
    double* host_slots_dev = nullptr;  // its device view (null: totals are copied back instead)

    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double setup_ms = 0.0;
    // the coarsest dense inverse runs on a second stream (one work-group): it overlaps the end of
    // the set-up and the start of the next solve, which waits for it before its first cycle
    hipStream_t side = nullptr;
    hipEvent_t ev_coarse = nullptr, ev_dense = nullptr;
    bool dense_pending = false;

    bool use_graphs = true;  // replay Krylov steps from captured graphs (needs a non-null stream)

    // optional per-kernel device timing of finest-level launches
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<TimedPair> pending;
    double kt_ms[64] = {};
    double kt_bytes[64] = {};
    long long kt_count[64] = {};
};

// Kernel identities for timing (finest level; float32 and float64 variants apart).
enum KId : int {
    KT_SMOOTH_FIRST = 0, KT_SMOOTH_HALF, KT_SMOOTH_HALF_DOT, KT_RESTRICT, KT_PROLONG_BLACK, KT_DIR_APPLY,
    KT_UPDATE_XR, KT_TRUE_RESIDUAL, KT_FIRST_RESTRICT, KT_PROLONG_HALF, KT_N
};
static const char* kt_name[KT_N] = {"smooth_first", "smooth_half", "smooth_half_dots", "residual_restrict",
                                    "prolong_black", "dir_apply", "update_xr", "true_residual", "first_restrict",
                                    "prolong_half"};

static hipEvent_t take_event(Handle* H)
{
    if (H->ev_used == H->ev_pool.size()) {
        hipEvent_t e;
        PP_HIP(hipEventCreate(&e));
        H->ev_pool.push_back(e);
    }
    return H->ev_pool[H->ev_used++];
}

// Brackets one launch with events when timing is on (id < 0: not timed).
struct TimeScope {
    Handle* H;
    int id;
    double bytes;
    hipEvent_t a = nullptr;
    TimeScope(Handle* h, int kid, double b) : H(h), id(kid), bytes(b)
    {
        if (H->timing && id >= 0) {
            a = take_event(H);
            PP_HIP(hipEventRecord(a, H->stream));
        }
    }
    ~TimeScope()
    {
        if (!a) return;
        try {
            hipEvent_t b = take_event(H);
            if (hipEventRecord(b, H->stream) == hipSuccess) H->pending.push_back({id, bytes, a, b});
        } catch (...) {
        }
    }
};

static void accumulate(Handle* H, const std::vector<TimedPair>& v)
{
    for (auto& p : v) {
        float ms = 0.f;
        PP_HIP(hipEventElapsedTime(&ms, p.a, p.b));
        H->kt_ms[p.id] += ms;
        H->kt_bytes[p.id] += p.bytes;
        H->kt_count[p.id] += 1;
    }
}

static void collect_timing(Handle* H)
{
    accumulate(H, H->pending);
    H->pending.clear();
    H->ev_used = 0;
}

static size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Walks the allocation plan; with base == nullptr it only counts bytes.
struct Planner {
    char* base;
    size_t off = 0;
    template <class T>
    T* take(size_t count)
    {
        size_t b = align_up(count * sizeof(T));
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += b;
        return p;
    }
};

static bool valid_cfg(const pp_config* cfg, std::string* why)
{
    if (!cfg) { if (why) *why = "null config"; return false; }
    if (cfg->nx < 2 || cfg->ny < 2 || cfg->nz < 2) { if (why) *why = "nx, ny, nz must be >= 2"; return false; }
    if (cfg->nz & 1) { if (why) *why = "nz must be even (red-black colouring across the periodic seam)"; return false; }
    if (!(cfg->h > 0.0) || !std::isfinite(cfg->h)) { if (why) *why = "h must be > 0"; return false; }
    if (!(cfg->tol > 0.0) || !std::isfinite(cfg->tol)) { if (why) *why = "tol must be > 0"; return false; }
    if (cfg->mode != PP_FP64 && cfg->mode != PP_FP32_REFINED) { if (why) *why = "unknown mode"; return false; }
    if (cfg->omega < 0.0 || cfg->omega >= 2.0 || !std::isfinite(cfg->omega)) { if (why) *why = "omega must be in [0, 2)"; return false; }
    if ((cfg->flags & PP_FLAG_MG_SOLVER) && cfg->mode != PP_FP64) { if (why) *why = "the multigrid-solver form is float64 only"; return false; }
    if ((cfg->flags & PP_FLAG_W_CYCLE) && !(cfg->flags & PP_FLAG_MG_SOLVER)) { if (why) *why = "W-cycles need the multigrid-solver form"; return false; }
    if (cfg->flags & ~(PP_FLAG_MG_SOLVER | PP_FLAG_W_CYCLE)) { if (why) *why = "unknown flag bits"; return false; }
    // 32-bit cell indices: the largest index plus one plane stride (a z-neighbour
    // read) must fit in an int
    if ((size_t)cfg->nx * cfg->ny * cfg->nz + (size_t)cfg->nx * cfg->ny > (size_t)INT_MAX) {
        if (why) *why = "grid too large (32-bit cell indices)";
        return false;
    }
    {
        Geo g = geo(cfg->nx, cfg->ny, cfg->nz);
        size_t most = (size_t)g.grid.x * g.grid.y * g.grid.z;
        for (int b : {8, 16, 32, 64}) {
            MGeo m = mgeo(cfg->nx, cfg->ny, cfg->nz, b);
            most = std::max(most, (size_t)m.grid.x * m.grid.y * m.grid.z);
        }
        // a reducing overlapped launch may use the whole partials buffer
        const MGeo o = ovl_geo(cfg->nx, cfg->ny, cfg->nz, kMaxPartialBlocks);
        if ((size_t)o.grid.x * o.grid.y * o.grid.z > (size_t)kMaxPartialBlocks) {
            if (why) *why = "cross-section too large for the overlapped-tile launches";
            return false;
        }
        if (most > (size_t)kMaxRedBlocks) {
            if (why) *why = "cross-section too large (more than 2048 thread tiles per plane)";
            return false;
        }
    }
    return true;
}

static void levels_of(const pp_config& cfg, std::vector<int>& nx, std::vector<int>& ny, std::vector<int>& nz)
{
    nx = {cfg.nx};
    ny = {cfg.ny};
    nz = {cfg.nz};
    while ((int)nx.size() < kMaxLev) {
        int a = nx.back(), b = ny.back(), c = nz.back();
        size_t n = (size_t)a * b * c;
        if (n <= (size_t)kDenseMax || (a & 1) || (b & 1) || (c & 3)) break;
        nx.push_back(a / 2);
        ny.push_back(b / 2);
        nz.push_back(c / 2);
    }
}

// Whether every pass on the finest level forms its face weights from the
// density (the plane-marching kernels with density weights): the level then
// keeps no stored weights, and the set-up forms its 1/D and the first coarse
// level's weights from the density directly.
static bool weights_from_density(const Params& prm) { return prm.march && prm.rho; }

// Lays out (or counts) every device array of a handle.
static size_t plan(Handle* H, const pp_config& cfg, char* base)
{
    Planner P{base};
    std::vector<int> nx, ny, nz;
    levels_of(cfg, nx, ny, nz);
    const int nl = (int)nx.size();
    const bool fp64 = cfg.mode == PP_FP64;
    const size_t n0 = (size_t)cfg.nx * cfg.ny * cfg.nz;
    auto nn = [&](int l) { return (size_t)nx[l] * ny[l] * nz[l]; };
    Params prm = H ? H->prm : Params{};

    // face weights of every level (level 0: beta_f) in float64, and in the
    // preconditioner's precision when that is float32; 1/D in that precision
    // (level 0 has none when every finest-level pass forms them from the density)
    std::vector<Level64> c64(nl);
    std::vector<Level32> c32(nl);
    const bool fine_rho = weights_from_density(prm);
    for (int l = 0; l < nl; ++l) {
        const bool stored = l > 0 || !fine_rho;
        if (stored) {
            c64[l].wx = P.take<double>(nn(l));
            c64[l].wy = P.take<double>(nn(l));
            c64[l].wz = P.take<double>(nn(l));
        }
        if (fp64) c64[l].invd = P.take<double>(nn(l));
        if (!fp64) {
            if (stored) {
                c32[l].wx = P.take<float>(nn(l));
                c32[l].wy = P.take<float>(nn(l));
                c32[l].wz = P.take<float>(nn(l));
            }
            c32[l].invd = P.take<float>(nn(l));
            if (l >= 1 && prm.hw && (long)nn(l) > prm.hwmin) {
                c32[l].hx = P.take<unsigned short>(nn(l));
                c32[l].hy = P.take<unsigned short>(nn(l));
                c32[l].hz = P.take<unsigned short>(nn(l));
            }
        }
    }
    const size_t nd = nn(nl - 1);
    double* M64 = nullptr;
    float* M32 = nullptr;
    if (nl > 1 && nd <= (size_t)kDenseMax) {
        M64 = P.take<double>(nd * nd);
        M32 = P.take<float>(nd * nd);
    }
    double* f64 = P.take<double>(n0);
    double* r64 = P.take<double>(n0);
    double* x64 = P.take<double>(n0);
    double* q64 = P.take<double>(n0);
    double* d_a = P.take<double>(n0);
    double* d_b = P.take<double>(n0);
    float* r32 = fp64 ? nullptr : P.take<float>(n0);
    double* rho64 = P.take<double>(n0);
    float* rho32 = fp64 ? nullptr : P.take<float>(n0);

    auto make_h = [&](auto tag, auto& Hh, bool alloc) {
        using T = decltype(tag);
        Hh.L.assign(nl, Lev<T>{});
        for (int l = 0; l < nl; ++l) {
            Lev<T>& V = Hh.L[l];
            V.nx = nx[l]; V.ny = ny[l]; V.nz = nz[l]; V.n = nn(l);
            V.kcyc = (l >= 1 && l <= prm.kmax && l < nl - 1 && V.n > (size_t)prm.kmin);
            if (!alloc) continue;
            if (l > 0) V.rhs = P.template take<T>(V.n);
            V.c = P.template take<T>(V.n);
            if (l < nl - 1) V.c2 = P.template take<T>(V.n);
            if (prm.gamma == 2 && l >= 1 && l < nl - 1) {
                V.w1 = P.template take<T>(V.n);
                V.rr = P.template take<T>(V.n);
            }
            if (V.kcyc) {
                if constexpr (std::is_same_v<T, float>) V.rhs2 = P.template take<T>(V.n);
                V.xk = P.template take<T>(V.n);
                V.d = V.d_a = P.template take<T>(V.n);
                V.d2 = V.d_b = P.template take<T>(V.n);
                V.q = P.template take<T>(V.n);
            }
        }
        if (fp64) { if constexpr (std::is_same_v<T, double>) Hh.Minv = M64; }
        else { if constexpr (std::is_same_v<T, float>) Hh.Minv = M32; }
        Hh.nd = (nl > 1 && nd <= (size_t)kDenseMax) ? (int)nd : 0;
    };
    Hier<double> h64;
    Hier<float> h32;
    make_h(double{}, h64, fp64);
    make_h(float{}, h32, !fp64);
    // the finest cycle reads the Krylov residual
    if (fp64) h64.L[0].rhs = r64;
    else h32.L[0].rhs = r32;
    double* partials = P.take<double>((size_t)kMaxPartialBlocks * kMaxRed);
    double* slots = P.take<double>(kSlots);

    if (H && base) {
        H->lnx = nx; H->lny = ny; H->lnz = nz; H->nlev = nl;
        H->c64 = c64; H->c32 = c32;
        H->M64 = M64; H->M32 = M32;
        H->f64 = f64; H->r64 = r64; H->x64 = x64; H->q64 = q64; H->r32 = r32;
        H->rho64 = rho64; H->rho32 = rho32;
        H->d = H->d_a = d_a; H->d2 = H->d_b = d_b;
        H->partials = partials; H->slots = slots;
        // operator views
        for (int l = 0; l < nl; ++l) {
            h64.L[l].v = LevelView<double>{nx[l], ny[l], nz[l], c64[l].wx, c64[l].wy, c64[l].wz, c64[l].invd};
            h32.L[l].v = LevelView<float>{nx[l], ny[l], nz[l], c32[l].wx, c32[l].wy, c32[l].wz, c32[l].invd};
            h32.L[l].v.hwx = c32[l].hx;
            h32.L[l].v.hwy = c32[l].hy;
            h32.L[l].v.hwz = c32[l].hz;
        }
        if (prm.rho) {
            h64.L[0].v.rho = rho64;
            h32.L[0].v.rho = rho32;
        }
        auto make_tail = [&](auto& Hh) {
            Hh.tail = -1;
            if (!prm.tail || nl < 2) return;
            // levels that fit: the first at most kTailMaxCells with even nx, the later
            // ones (iterates and operators in LDS) at most kTailSmallCells together
            int t = nl - 1;
            size_t later = 0;
            while (t - 1 >= 1 && !Hh.L[t - 1].kcyc && Hh.L[t - 1].n <= (size_t)prm.tail_max &&
                   (Hh.L[t - 1].nx % 2) == 0 && later + Hh.L[t].n <= (size_t)kTailSmallCells) {
                later += Hh.L[t].n;
                --t;
            }
            if (t == nl - 1 || t <= prm.kmax || nl - t > kTailMaxLev) return;  // need at least two levels
            Hh.tail = t;
            auto& D = Hh.td;
            D.nlev = nl - t;
            int off = 0;
            for (int l = t; l < nl; ++l) {
                auto& V = Hh.L[l];
                D.L[l - t].v = V.v;
                D.L[l - t].rhs = V.rhs;
                D.L[l - t].c = V.c;
                D.L[l - t].n = (int)V.n;
                D.L[l - t].off = off;
                if (l > t) off += (int)V.n;
            }
            // the first level joins the later ones in LDS when it fits beside them
            D.lds0 = (size_t)off + Hh.L[t].n <= (size_t)kTailSmallCells;
            D.off0 = off;
            D.Minv = Hh.Minv;
            D.nd = Hh.nd;
            D.wc = prm.wc;
            D.omega = prm.omega;
            D.nu = prm.nuv > 0 ? prm.nuv : prm.nuc;
            D.coarse_sweeps = prm.coarse_sweeps;
        };
        if (fp64) make_tail(h64);
        else make_tail(h32);
        H->h64 = h64;
        H->h32 = h32;
    }
    return P.off;
}

// ---------------------------------------------------------------- small helpers

static Reduce red(Handle* H, int s0, int s1 = 0, int s2 = 0, int s3 = 0)
{
    Reduce R;
    R.partials = H->partials;
    R.out = H->slots;
    R.slot[0] = s0; R.slot[1] = s1; R.slot[2] = s2; R.slot[3] = s3;
    return R;
}
// The same for totals the host reads next: the finishing kernel also writes
// them into the mapped host slots (see fetch_slots).
static Reduce red_host(Handle* H, int s0, int s1 = 0, int s2 = 0)
{
    Reduce R = red(H, s0, s1, s2);
    R.host = H->host_slots_dev;
    return R;
}

static Coefs coef(Handle* H, int num, int den, double sign) { return Coefs{H->slots, num, den, sign}; }

// Work of an entry point runs on the handle's stream, after everything queued
// on the caller's stream before the call, and the caller's stream waits for it.
static void enter(Handle* H)
{
    PP_HIP(hipEventRecord(H->ev_in, H->user));
    PP_HIP(hipStreamWaitEvent(H->stream, H->ev_in, 0));
}
static void leave(Handle* H)
{
    PP_HIP(hipEventRecord(H->ev_out, H->stream));
    PP_HIP(hipStreamWaitEvent(H->user, H->ev_out, 0));
}

static void check_launch()
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw Fail(PP_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
}

// Completes a reducing launch with the given grid: its nv totals land in the slots.
static void finish(Handle* H, const Reduce& R, const dim3& grid, int nv)
{
    k_reduce_finish<<<1, kBlock, 0, H->stream>>>(R, (int)(grid.x * grid.y * grid.z), nv);
    check_launch();
}

static void read_slots(Handle* H, int first, int count)
{
    PP_HIP(hipMemcpyAsync(H->host_slots + first, H->slots + first, sizeof(double) * count, hipMemcpyDeviceToHost, H->stream));
    PP_HIP(hipStreamSynchronize(H->stream));
}

// Makes host_slots[first, first + count) current after a reduction made with
// red_host: waits for the stream (the finishing kernel wrote them into the
// mapped host slots), or copies them back when the slots are not mapped.
static void fetch_slots(Handle* H, int first, int count)
{
    if (H->host_slots_dev) PP_HIP(hipStreamSynchronize(H->stream));
    else read_slots(H, first, count);
}

static void write_slots(Handle* H, int first, const double* v, int count)
{
    for (int i = 0; i < count; ++i) H->host_slots[first + i] = v[i];
    PP_HIP(hipMemcpyAsync(H->slots + first, H->host_slots + first, sizeof(double) * count, hipMemcpyHostToDevice, H->stream));
}

// ---------------------------------------------------------------- multigrid cycle

template <class T>
static int kid(int id) { return id + (sizeof(T) == 4 ? 0 : 32); }

// The float64 finest-level operator (with the density when the plane-marching
// kernels derive the weights from it).
static LevelView<double> fine64(const Handle* H)
{
    LevelView<double> v{H->cfg.nx, H->cfg.ny, H->cfg.nz, H->c64[0].wx, H->c64[0].wy, H->c64[0].wz, nullptr};
    if (H->prm.rho) v.rho = H->rho64;
    return v;
}

// Arrays a pass reads for the face weights of a level: the density alone when
// the plane-marching kernels form them from it, else the three weight arrays.
template <class T>
static double weight_arrays(const Handle* H, const LevelView<T>& v)
{
    // in units of the view's precision: density 1, bfloat16 weights 3 halves, stored 3
    if (!H->prm.march) return 3.0;
    return v.rho ? 1.0 : (v.hwx ? 1.5 : 3.0);
}

// Whether a level smoothed once runs its passes as overlapped-tile launches.
static bool fused(const Handle* H, size_t prec, size_t n)
{
    return H->prm.march && ((long)n >= H->prm.fbig || (long)n <= H->prm.fsmall) &&
           (H->prm.fuse == 2 || (H->prm.fuse == 1 && prec == 4));
}

// 1/D arrays read by a half-sweep or prolongation: the march kernels divide by
// the stencil's own diagonal, the per-cell kernels read 1/D.
static double invd_arrays(const Handle* H) { return H->prm.march ? 0.0 : 1.0; }

template <int M>
using WmC = std::integral_constant<int, M>;
// Calls f(WmC<m>{}) with the source m of the view's face weights for the
// march kernels: the density, bfloat16 copies, or the stored arrays.
template <class T, class F>
static void with_rho(const LevelView<T>& v, F&& f)
{
    if (v.rho) f(WmC<kWRho>{});
    else if constexpr (std::is_same_v<T, float>) {
        if (v.hwx) f(WmC<kWHalf>{});
        else f(WmC<kWStored>{});
    } else {
        f(WmC<kWStored>{});
    }
}

// XCD-aware tile order for a march launch on a level of this size (see tile_of_block).
template <class T>
static int xcd_of(const Handle* H, const LevelView<T>& v)
{
    const size_t n = (size_t)v.nx * v.ny * v.nz;
    return H->prm.xcd == 1 || (H->prm.xcd == 2 && n < ((size_t)H->cfg.nx * H->cfg.ny * H->cfg.nz));
}

// Geometry of a march launch on view v (block size as in kMarchThreads).
template <class T>
static MGeo march_geo(const Handle* H, const LevelView<T>& v, int bx_max, bool even_k = false)
{
    if (v.rho && kMarchThreads<T, true> != kBlock)
        return mgeo(v.nx, v.ny, v.nz, bx_max, even_k, H->prm.fblocks, kMarchThreads<T, true>);
    return mgeo(v.nx, v.ny, v.nz, bx_max, even_k, H->prm.mblocks, kBlock);
}

// Row-wave geometry of a finest-level float64 pass (cpt = cells per lane), or
// cpt = 0 when the row-wave kernels do not apply: they need the density-formed
// weights and a row of 64, 128, 192 or 256 cells.
struct RwGeo {
    dim3 grid, block;
    int kper = 0, cpt = 0, rows = 8, wpr = 1;  // wpr: wavefronts per row
    int xcd = 0;                               // XCD-aware band order
};
// z split of a row-wave launch of gy bands: about max_blocks blocks of kper
// planes (kper even when the pass pairs planes).  With the XCD-aware band order
// the number of z ranges is rounded down to a multiple of 8 where that is
// possible, so that the block count is one (the order needs it; else the
// blocks keep the plain order) and each XCD runs a contiguous run of bands:
// the ring and halo rows a band shares with its neighbours then come into that
// XCD's L2 once.
static void rw_zsplit(int xcd, int gy, int nz, int max_blocks, bool even, int& gz, int& kper)
{
    gz = std::max(1, std::min(even ? nz / 2 : nz, max_blocks / gy));
    if (xcd && gz >= 8 && (gy & 7)) gz -= gz & 7;
    kper = (nz + gz - 1) / gz;
    if (even && (kper & 1)) ++kper;
    gz = (nz + kper - 1) / kper;
}

static RwGeo rw_geo(const Handle* H, const LevelView<double>& v)
{
    RwGeo g;
    if (!H->prm.rw || !H->prm.march || !v.rho || v.nx % 64 != 0 || v.nx > 256) return g;
    // a row over two wavefronts where the row is 128 or 256 cells
    const int wpr = (H->prm.rwsplit == 2 && v.nx % 128 == 0) ? 2 : 1;
    const int rows = wpr == 2 ? H->prm.rwsrows : H->prm.rwrows;
    const int xcd = wpr == 2 ? H->prm.rwsxcd : H->prm.rwxcd;
    const int gy = (v.ny + rows - 1) / rows;
    int gz, kper;
    rw_zsplit(xcd, gy, v.nz, wpr == 2 ? H->prm.rwsblocks : H->prm.rwblocks, false, gz, kper);
    if ((size_t)gy * gz > (size_t)kMaxPartialBlocks) return g;
    g.grid = dim3(1, gy, gz);
    g.block = dim3(64 * wpr, rows, 1);
    g.xcd = xcd;
    g.rows = rows;
    g.kper = kper;
    g.wpr = wpr;
    g.cpt = v.nx / (64 * wpr);
    return g;
}
// Row-wave geometry of a pass on a float32 level with bfloat16 weights, or cpt = 0.
template <class T>
static RwGeo rwc_geo(const Handle* H, const LevelView<T>& v)
{
    RwGeo g;
    if constexpr (std::is_same_v<T, float>) {
        if (!H->prm.rwc || !H->prm.march || !v.hwx || v.nx % 64 != 0 || v.nx > 256) return g;
        const int rows = H->prm.rwcrows;
        const int gy = (v.ny + rows - 1) / rows;
        int gz, kper;
        rw_zsplit(H->prm.rwcxcd, gy, v.nz, H->prm.rwcblocks, false, gz, kper);
        if ((size_t)gy * gz > (size_t)kMaxPartialBlocks) return g;
        g.grid = dim3(1, gy, gz);
        g.block = dim3(64, rows, 1);
        g.kper = kper;
        g.cpt = v.nx / 64;
        g.rows = rows;
        g.xcd = H->prm.rwcxcd;
    }
    return g;
}

// Calls f(BxC<cpt>{}, BxC<rows>{}) for the row-wave instantiations.
template <class F>
static void with_cpt(const RwGeo& g, F&& f)
{
    auto rows = [&](auto C) {
        if (g.rows == 4) f(C, BxC<4>{});
        else f(C, BxC<8>{});
    };
    switch (g.cpt) {
    case 1: rows(BxC<1>{}); break;
    case 2: rows(BxC<2>{}); break;
    case 3: rows(BxC<3>{}); break;
    default: rows(BxC<4>{}); break;
    }
}

// Calls f(BxC<cpt>{}, BxC<rows>{}, BxC<wpr>{}) for the finest-level float64
// row-wave instantiations: one wavefront per row as with_cpt, or a row over two
// wavefronts (cpt 1 or 2, rows 4, 6 or 8).
template <class F>
static void with_cpt_rw(const RwGeo& g, F&& f)
{
    if (g.wpr == 1) {
        with_cpt(g, [&](auto C, auto Y) { f(C, Y, BxC<1>{}); });
        return;
    }
    auto rows = [&](auto C) {
        if (g.rows == 4) f(C, BxC<4>{}, BxC<2>{});
        else if (g.rows == 6) f(C, BxC<6>{}, BxC<2>{});
        else f(C, BxC<8>{}, BxC<2>{});
    };
    if (g.cpt == 1) rows(BxC<1>{});
    else rows(BxC<2>{});
}

// Launchers: the plane-march kernels, or the per-column kernels when the march is off.

template <class T>
static void launch_first(Handle* H, const LevelView<T>& v, const T* f, T* x)
{
    const T om = (T)H->prm.omega;
    if constexpr (std::is_same_v<T, float>) {
        const RwGeo rg = rwc_geo(H, v);
        if (rg.cpt) {
            with_cpt(rg, [&](auto C, auto Y) {
                r_smooth_first<decltype(C)::value, decltype(Y)::value>
                    <<<rg.grid, rg.block, 0, H->stream>>>(v, f, x, rg.kper, rg.xcd, om);
            });
            check_launch();
            return;
        }
    }
    if (H->prm.march) {
        const MGeo g = march_geo(H, v, H->prm.mbx);
        with_bx(g.bx, [&](auto B) {
            with_rho(v, [&](auto R) {
                m_smooth_first<T, decltype(B)::value, decltype(R)::value><<<g.grid, g.block, 0, H->stream>>>(v, f, x, g.kper,
                                                                                                           xcd_of(H, v), om);
            });
        });
    } else {
        const Geo g = geo(v.nx, v.ny, v.nz);
        k_smooth_first<T><<<g.grid, g.block, 0, H->stream>>>(v, f, x, g.kper, om);
    }
    check_launch();
}

// Launchers of reducing kernels return the grid; the caller completes the
// reduction with finish() (outside any timed scope).
template <class T, int NDOT, class TQ>
static dim3 launch_half(Handle* H, const LevelView<T>& v, const T* f, T* x, int colour, const TQ* q, const Reduce& R)
{
    const T om = (T)H->prm.omega;
    if constexpr (std::is_same_v<T, float>) {
        const RwGeo rg = rwc_geo(H, v);
        if (rg.cpt) {
            with_cpt(rg, [&](auto C, auto Y) {
                r_smooth_half<decltype(C)::value, decltype(Y)::value, NDOT, TQ>
                    <<<rg.grid, rg.block, 0, H->stream>>>(v, f, x, colour, rg.kper, rg.xcd, q, R, om);
            });
            check_launch();
            return rg.grid;
        }
    }
    if (H->prm.march) {
        const MGeo g = march_geo(H, v, H->prm.mbx);
        with_bx(g.bx, [&](auto B) {
            with_rho(v, [&](auto W) {
                m_smooth_half<T, decltype(B)::value, decltype(W)::value, NDOT, TQ>
                    <<<g.grid, g.block, 0, H->stream>>>(v, f, x, colour, g.kper, xcd_of(H, v), q, R, om);
            });
        });
        check_launch();
        return g.grid;
    }
    const Geo g = geo(v.nx, v.ny, v.nz);
    k_smooth_half<T, NDOT, TQ><<<g.grid, g.block, 0, H->stream>>>(v, f, x, colour, g.kper, q, R, om);
    check_launch();
    return g.grid;
}

template <class T>
static void launch_restrict(Handle* H, const LevelView<T>& v, const T* f, const T* x, T* rc)
{
    if (H->prm.march) {
        const MGeo g = march_geo(H, v, std::min(H->prm.mbx, 32), true);
        with_bx_le32(g.bx, [&](auto B) {
            with_rho(v, [&](auto R) {
                m_residual_restrict<T, decltype(B)::value, decltype(R)::value>
                    <<<g.grid, g.block, 0, H->stream>>>(v, f, x, rc, g.kper, xcd_of(H, v));
            });
        });
    } else {
        const Geo g = geo(v.nx / 2, v.ny / 2, v.nz / 2);
        k_residual_restrict<T><<<g.grid, g.block, 0, H->stream>>>(v, f, x, rc, v.nx / 2, v.ny / 2, v.nz / 2, g.kper);
    }
    check_launch();
}

// Row-wave geometry of a fused float32 finest-level pass: bands of rows - 2
// own rows (plus a ring row on each side), z ranges of an even number of
// planes; cpt = 0 when it does not apply (density-formed weights, nx 128 or 256).
static RwGeo rwf_geo(const Handle* H, const LevelView<float>& v, int max_blocks)
{
    RwGeo g;
    if (!H->prm.rwf || !H->prm.march || !v.rho || (v.nx != 128 && v.nx != 256)) return g;
    const int rows = H->prm.rwfrows, sy = rows - 2;
    const int gy = (v.ny + sy - 1) / sy;
    int gz, kper;
    rw_zsplit(H->prm.rwfxcd, gy, v.nz, max_blocks, true, gz, kper);
    if ((size_t)gy * gz > (size_t)kMaxPartialBlocks) return g;
    g.grid = dim3(1, gy, gz);
    g.block = dim3(64, rows, 1);
    g.kper = kper;
    g.cpt = v.nx / 64;
    g.rows = rows;
    return g;
}
template <class F>
static void with_cpt_even(const RwGeo& g, F&& f)
{
    auto rows = [&](auto C) {
        if (g.rows == 16) f(C, BxC<16>{});
        else if (g.rows == 12) f(C, BxC<12>{});
        else f(C, BxC<8>{});
    };
    if (g.cpt == 2) rows(BxC<2>{});
    else rows(BxC<4>{});
}

// First sweep from zero and restriction of its residual in one launch (a
// level smoothed once before the coarse correction).
template <class T>
static void launch_first_restrict(Handle* H, const LevelView<T>& v, const T* f, T* x, T* rc)
{
    if constexpr (std::is_same_v<T, float>) {
        const RwGeo rg = rwf_geo(H, v, H->prm.rwfblocks);
        if (rg.cpt) {
            with_cpt_even(rg, [&](auto C, auto Y) {
                r_first_restrict<decltype(C)::value, decltype(Y)::value>
                    <<<rg.grid, rg.block, 0, H->stream>>>(v, f, x, rc, rg.kper, H->prm.rwfxcd, (T)H->prm.omega);
            });
            check_launch();
            return;
        }
    }
    const MGeo g = ovl_geo(v.nx, v.ny, v.nz, H->prm.oblocks);
    const int xcd = H->prm.oxcd < 0 ? xcd_of(H, v) : H->prm.oxcd;
    with_rho(v, [&](auto R) {
        m_first_restrict<T, decltype(R)::value>
            <<<g.grid, g.block, 0, H->stream>>>(v, f, x, rc, g.kper, xcd, (T)H->prm.omega);
    });
    check_launch();
}

// Prolongation, black update and the red half-sweep after it in one launch (a
// level smoothed once after the coarse correction); NDOT dots as in launch_half.
template <class T, int NDOT, class TQ>
static dim3 launch_prolong_half(Handle* H, const LevelView<T>& v, const T* f, const T* x, const T* e, T wc, T* z,
                                const TQ* q, const Reduce& R)
{
    if constexpr (std::is_same_v<T, float>) {
        const RwGeo rg = rwf_geo(H, v, H->prm.rwfblocks);
        if (rg.cpt) {
            with_cpt_even(rg, [&](auto C, auto Y) {
                r_prolong_half<decltype(C)::value, decltype(Y)::value, NDOT, TQ><<<rg.grid, rg.block, 0, H->stream>>>(
                    v, f, x, e, wc, z, q, R, rg.kper, H->prm.rwfxcd, (T)H->prm.omega);
            });
            check_launch();
            return rg.grid;
        }
    }
    // a reducing launch writes one partial per block: at most kMaxPartialBlocks blocks
    const MGeo g = ovl_geo(v.nx, v.ny, v.nz, NDOT > 0 ? std::min(H->prm.oblocks, kMaxPartialBlocks) : H->prm.oblocks);
    if (NDOT > 0 && (size_t)g.grid.x * g.grid.y * g.grid.z > (size_t)kMaxPartialBlocks)
        throw Fail(PP_ERR_INVALID, "cross-section too large for a reducing overlapped-tile launch");
    const int xcd = H->prm.oxcd < 0 ? xcd_of(H, v) : H->prm.oxcd;
    with_rho(v, [&](auto W) {
        m_prolong_half<T, decltype(W)::value, NDOT, TQ>
            <<<g.grid, g.block, 0, H->stream>>>(v, f, x, e, wc, z, q, R, g.kper, xcd, (T)H->prm.omega);
    });
    check_launch();
    return g.grid;
}

template <class T>
static void launch_prolong_black(Handle* H, const LevelView<T>& v, const T* f, const T* x, const T* e, T wc, T* y)
{
    const T om = (T)H->prm.omega;
    if constexpr (std::is_same_v<T, float>) {
        const RwGeo rg = rwc_geo(H, v);
        if (rg.cpt) {
            with_cpt(rg, [&](auto C, auto Y) {
                r_prolong_black<decltype(C)::value, decltype(Y)::value>
                    <<<rg.grid, rg.block, 0, H->stream>>>(v, f, x, e, wc, y, rg.kper, rg.xcd, om);
            });
            check_launch();
            return;
        }
    }
    if (H->prm.march) {
        const MGeo g = march_geo(H, v, H->prm.mbx);
        with_bx(g.bx, [&](auto B) {
            with_rho(v, [&](auto R) {
                m_prolong_black<T, decltype(B)::value, decltype(R)::value>
                    <<<g.grid, g.block, 0, H->stream>>>(v, f, x, e, wc, y, g.kper, xcd_of(H, v), om);
            });
        });
    } else {
        const Geo g = geo(v.nx, v.ny, v.nz);
        k_prolong_black<T><<<g.grid, g.block, 0, H->stream>>>(v, f, x, e, wc, y, g.kper, om);
    }
    check_launch();
}

// FINE: the finest level's step (dot <d,q> only; x += aprev * d_old after the first step).
template <class T, class TZ, bool FINE = false>
static dim3 launch_dir(Handle* H, const LevelView<T>& v, const TZ* z, const T* dold, T* dnew, T* q, const T* r, T* x,
                       Coefs beta, int use_beta, Coefs mean, int use_mean, Coefs aprev, const Reduce& R)
{
    if constexpr (!FINE && std::is_same_v<T, float> && std::is_same_v<TZ, float>) {
        const RwGeo rg = rwc_geo(H, v);
        if (rg.cpt) {
            with_cpt(rg, [&](auto C, auto Y) {
                constexpr int CPT = decltype(C)::value, BY = decltype(Y)::value;
                if (use_beta)
                    r_dir_apply_f32<CPT, BY, true><<<rg.grid, rg.block, 0, H->stream>>>(
                        v, z, dold, dnew, q, r, beta, mean, use_mean, rg.kper, rg.xcd, R);
                else
                    r_dir_apply_f32<CPT, BY, false><<<rg.grid, rg.block, 0, H->stream>>>(
                        v, z, dold, dnew, q, r, beta, mean, use_mean, rg.kper, rg.xcd, R);
            });
            check_launch();
            return rg.grid;
        }
    }
    if constexpr (FINE && std::is_same_v<T, double>) {
        RwGeo rg = H->prm.rwdir ? rw_geo(H, v) : RwGeo{};
        if (H->prm.rwdir == 2 && rg.wpr == 1) rg.cpt = 0;  // one wavefront per row: the tiles are faster
        if (rg.cpt) {
            with_cpt_rw(rg, [&](auto C, auto Y, auto P) {
                constexpr int CPT = decltype(C)::value, BY = decltype(Y)::value, WPR = decltype(P)::value;
                if (use_beta)
                    r_dir_apply<CPT, BY, TZ, true, FINE, WPR><<<rg.grid, rg.block, 0, H->stream>>>(
                        v, z, dold, dnew, q, r, x, beta, mean, use_mean, aprev, rg.kper, rg.xcd, R);
                else
                    r_dir_apply<CPT, BY, TZ, false, FINE, WPR><<<rg.grid, rg.block, 0, H->stream>>>(
                        v, z, dold, dnew, q, r, x, beta, mean, use_mean, aprev, rg.kper, rg.xcd, R);
            });
            check_launch();
            return rg.grid;
        }
    }
    if (H->prm.march) {
        const MGeo g = march_geo(H, v, H->prm.mbx);
        with_bx(g.bx, [&](auto B) {
            with_rho(v, [&](auto W) {
                constexpr int BX = decltype(B)::value;
                constexpr int WM = decltype(W)::value;
                if (use_beta)
                    m_dir_apply<T, BX, WM, TZ, true, FINE><<<g.grid, g.block, 0, H->stream>>>(
                        v, z, dold, dnew, q, r, x, beta, mean, use_mean, aprev, g.kper, xcd_of(H, v), R);
                else
                    m_dir_apply<T, BX, WM, TZ, false, FINE><<<g.grid, g.block, 0, H->stream>>>(
                        v, z, dold, dnew, q, r, x, beta, mean, use_mean, aprev, g.kper, xcd_of(H, v), R);
            });
        });
        check_launch();
        return g.grid;
    }
    const Geo g = geo(v.nx, v.ny, v.nz);
    k_dir_apply<T, TZ, FINE><<<g.grid, g.block, 0, H->stream>>>(v, z, dold, dnew, q, r, x, beta, use_beta, mean, use_mean, aprev,
                                                                g.kper, R);
    check_launch();
    return g.grid;
}

template <class T, class TQ>
static void smooth_half(Handle* H, Lev<T>& V, bool fine, const T* f, T* x, int colour, int ndot, const TQ* q, int l)
{
    Reduce R = red(H, lslot(l, S_SUMZ), lslot(l, S_ZQ), H->zr_slot, H->fsum_slot);
    dim3 grid;
    {
        // reads x, f and the weights (or the density; the per-cell kernels also 1/D); writes one
        // colour (and reads q for the dot)
        TimeScope ts(H, fine ? kid<T>(ndot ? KT_SMOOTH_HALF_DOT : KT_SMOOTH_HALF) : -1,
                     (double)V.n * ((2.5 + invd_arrays(H) + weight_arrays(H, V.v)) * sizeof(T) +
                                    (ndot >= 2 ? sizeof(TQ) : 0)));
        if (ndot == 0) grid = launch_half<T, 0, TQ>(H, V.v, f, x, colour, q, R);
        else if (ndot == 1) grid = launch_half<T, 1, TQ>(H, V.v, f, x, colour, q, R);
        else if (ndot == 2) grid = launch_half<T, 2, TQ>(H, V.v, f, x, colour, q, R);
        else grid = launch_half<T, 4, TQ>(H, V.v, f, x, colour, q, R);
    }
    if (ndot > 0) finish(H, R, grid, ndot);
}

template <class T>
static T* kcycle(Handle* H, Hier<T>& Hh, int l);
template <class T>
static T* second_visit(Handle* H, Hier<T>& Hh, int m, T* e);

// Red-black sweeps of level l before and after its coarse correction.
template <class T>
static int sweeps_of(const Handle* H, const Lev<T>& V, int l)
{
    return l == 0                                             ? H->prm.nu0
           : (l == 1 && H->prm.nu1 > 0)                       ? H->prm.nu1
           : (V.kcyc && l >= 2 && H->prm.nuk2 > 0)            ? H->prm.nuk2
           : (!V.kcyc && l > H->prm.kmax && H->prm.nuv > 0)   ? H->prm.nuv
                                                              : H->prm.nuc;
}

// A K-cycle step's residual formed inside its cycle's first pass: f = r - alpha q
// from the previous step's r and q, stored into out (see kcycle).
template <class T>
struct Fold {
    const T* r;
    const T* q;
    T* out;
    Coefs alpha;
};

// The first sweep from zero on fd's residual (row-wave float32 levels: see kfold_ok).
template <class T>
static void launch_first_fold(Handle* H, const LevelView<T>& v, const Fold<T>& fd, T* x)
{
    if constexpr (std::is_same_v<T, float>) {
        const RwGeo rg = rwc_geo(H, v);
        if (rg.cpt) {
            with_cpt(rg, [&](auto C, auto Y) {
                r_smooth_first_r<decltype(C)::value, decltype(Y)::value><<<rg.grid, rg.block, 0, H->stream>>>(
                    v, fd.r, fd.q, fd.alpha, fd.out, x, rg.kper, rg.xcd, (float)H->prm.omega);
            });
            check_launch();
            return;
        }
    }
    throw Fail(PP_ERR_INVALID, "folded K-cycle step on a level without row-wave passes");
}

// Down leg of a cycle at level l: nu red-black sweeps of K x = f from a zero
// guess into x, then the residual f - K x summed over the 8 children of each
// coarse cell into rc (one overlapped-tile launch on a fused level).  With fold
// the first sweep forms f itself (f == fold->out).
template <class T>
static void cycle_pre(Handle* H, Lev<T>& V, int l, int nu, const T* f, T* x, T* rc, const Fold<T>* fold = nullptr)
{
    const bool fine = (l == 0);
    if (!fold && nu == 1 && fused(H, sizeof(T), V.n)) {
        // reads f, 1/D and the weights (or the density); writes x and the coarse right-hand side
        TimeScope ts(H, fine ? kid<T>(KT_FIRST_RESTRICT) : -1, (double)V.n * sizeof(T) * (3.125 + weight_arrays(H, V.v)));
        launch_first_restrict<T>(H, V.v, f, x, rc);
        return;
    }
    {
        // reads f, 1/D and the weights (or the density); writes x
        TimeScope ts(H, fine ? kid<T>(KT_SMOOTH_FIRST) : -1, (double)V.n * sizeof(T) * (3.0 + weight_arrays(H, V.v)));
        if (fold) launch_first_fold<T>(H, V.v, *fold, x);  // f is fold->out, which this pass writes
        else launch_first<T>(H, V.v, f, x);
    }
    for (int s = 1; s < nu; ++s) {
        smooth_half(H, V, fine, f, x, 0, 0, (const T*)nullptr, l);
        smooth_half(H, V, fine, f, x, 1, 0, (const T*)nullptr, l);
    }
    // reads x, f and the weights (or the density); writes the coarse right-hand side
    TimeScope ts(H, fine ? kid<T>(KT_RESTRICT) : -1, (double)V.n * sizeof(T) * (2.125 + weight_arrays(H, V.v)));
    launch_restrict<T>(H, V.v, f, x, rc);
}

// Up leg of a cycle at level l: y = x + wc P e (injection), then nu sweeps
// (black, then red) of K y = f, the first black half-sweep fused with the
// prolongation (and, on a fused level, the red one too).  ndot: 0 none,
// 1 sum(y), 2 sum(y) and <y, q>, 4 also <y, f> and sum(f) (into H->zr_slot and
// H->fsum_slot), reduced on the last half-sweep into level l's slots.  Returns y.
template <class T, class TQ>
static T* cycle_post(Handle* H, Lev<T>& V, int l, int nu, const T* f, const T* x, const T* e, T wc, T* y, int ndot,
                     const TQ* q)
{
    const bool fine = (l == 0);
    if (nu == 1 && H->prm.pfuse && fused(H, sizeof(T), V.n)) {
        // reads x, f, the weights (or the density), the coarse correction and q for the dot;
        // writes z
        const Reduce R = red(H, lslot(l, S_SUMZ), lslot(l, S_ZQ), H->zr_slot, H->fsum_slot);
        dim3 grid;
        {
            TimeScope ts(H, fine ? kid<T>(KT_PROLONG_HALF) : -1,
                         (double)V.n * ((3.125 + weight_arrays(H, V.v)) * sizeof(T) + (ndot >= 2 ? sizeof(TQ) : 0)));
            if (ndot == 0) grid = launch_prolong_half<T, 0, TQ>(H, V.v, f, x, e, wc, y, q, R);
            else if (ndot == 1) grid = launch_prolong_half<T, 1, TQ>(H, V.v, f, x, e, wc, y, q, R);
            else if (ndot == 2) grid = launch_prolong_half<T, 2, TQ>(H, V.v, f, x, e, wc, y, q, R);
            else grid = launch_prolong_half<T, 4, TQ>(H, V.v, f, x, e, wc, y, q, R);
        }
        if (ndot > 0) finish(H, R, grid, ndot);
        return y;
    }
    {
        // reads x, f, the weights (or the density) and the coarse correction (the per-cell
        // kernels also 1/D); writes y
        TimeScope ts(H, fine ? kid<T>(KT_PROLONG_BLACK) : -1,
                     (double)V.n * sizeof(T) * (3.125 + invd_arrays(H) + weight_arrays(H, V.v)));
        launch_prolong_black<T>(H, V.v, f, x, e, wc, y);
    }
    for (int s = 0; s < nu; ++s) {
        if (s > 0) smooth_half(H, V, fine, f, y, 1, 0, (const T*)nullptr, l);
        smooth_half(H, V, fine, f, y, 0, (s == nu - 1) ? ndot : 0, q, l);
    }
    return y;
}


// One multigrid cycle at level l for right-hand side f; returns the buffer holding
// the result.  ndot: 0 none, 1 sum(z), 2 sum(z) and <z, q>, 4 also <z, f> and
// sum(f) (into H->zr_slot and H->fsum_slot), reduced on the last half-sweep into
// level l's slots.
template <class T, class TQ = T>
static T* mgcycle(Handle* H, Hier<T>& Hh, int l, const T* f, int ndot, const TQ* q, const Fold<T>* fold = nullptr)
{
    Lev<T>& V = Hh.L[l];
    const bool fine = (l == 0);
    const int last = (int)Hh.L.size() - 1;
    if (l == Hh.tail && l > 0) {
        if (Hh.td.lds0) k_tail_vcycle<T, true><<<1, kTailThreads, 0, H->stream>>>(Hh.td);
        else k_tail_vcycle<T, false><<<1, kTailThreads, 0, H->stream>>>(Hh.td);
        check_launch();
        return V.c;
    }
    if (l == last) {
        if (l > 0 && Hh.nd > 0) {
            k_dense_apply<T><<<1, kBlock, 0, H->stream>>>(Hh.nd, Hh.Minv, f, V.c);
            check_launch();
        } else {
            // symmetric block of red-black sweeps (also the whole cycle when the
            // finest level cannot be coarsened)
            {
                TimeScope ts(H, fine ? kid<T>(KT_SMOOTH_FIRST) : -1, (double)V.n * sizeof(T) * (3.0 + weight_arrays(H, V.v)));
                launch_first<T>(H, V.v, f, V.c);
            }
            const int ns = H->prm.coarse_sweeps;
            for (int s = 1; s < ns; ++s) {
                smooth_half(H, V, fine, f, V.c, 0, 0, (const T*)nullptr, l);
                smooth_half(H, V, fine, f, V.c, 1, 0, (const T*)nullptr, l);
            }
            for (int s = 0; s < ns; ++s) {
                smooth_half(H, V, fine, f, V.c, 1, 0, (const T*)nullptr, l);
                smooth_half(H, V, fine, f, V.c, 0, (s == ns - 1) ? ndot : 0, q, l);
            }
        }
        return V.c;
    }
    const int nu = sweeps_of(H, V, l);
    Lev<T>& C = Hh.L[l + 1];
    cycle_pre(H, V, l, nu, f, V.c, C.rhs, fold);
    T* e;
    T wc;
    if (C.kcyc) {
        e = kcycle(H, Hh, l + 1);
        wc = T(1);
    } else {
        e = mgcycle(H, Hh, l + 1, C.rhs, 0, (const T*)nullptr);
        wc = (T)H->prm.wc;
        if (H->prm.gamma == 2 && C.w1 && l + 1 != Hh.tail) e = second_visit(H, Hh, l + 1, e);
    }
    return cycle_post(H, V, l, nu, f, V.c, e, wc, V.c2, ndot, q);
}

// W-cycle: the second stationary visit of level m, e <- e + M (f_m - K_m e),
// with M one cycle from level m (returns the level's w1 buffer).
template <class T>
static T* second_visit(Handle* H, Hier<T>& Hh, int m, T* e)
{
    Lev<T>& C = Hh.L[m];
    const Coefs one = coef(H, G_ONE, -1, 1.0);
    const dim3 lg = lin_grid(C.n);
    k_update_xr<T><<<lg, kBlock, 0, H->stream>>>((int)C.n, C.w1, e, (T*)nullptr, (const T*)nullptr, one, 1, 1, 0,
                                                 red(H, G_FN2), (float*)nullptr, 1);
    check_launch();
    const Geo g = geo(C.nx, C.ny, C.nz);
    k_residual<T><<<g.grid, g.block, 0, H->stream>>>(C.v, C.rhs, C.w1, C.rr, g.kper);
    check_launch();
    T* e2 = mgcycle(H, Hh, m, C.rr, 0, (const T*)nullptr);
    k_update_xr<T><<<lg, kBlock, 0, H->stream>>>((int)C.n, C.w1, e2, (T*)nullptr, (const T*)nullptr, one, 0, 1, 0,
                                                 red(H, G_FN2), (float*)nullptr, 1);
    check_launch();
    return C.w1;
}

template <class T>
static void dir_apply(Handle* H, Lev<T>& V, bool fine, const T* z, int it, int l, bool mean)
{
    const int dq_prev = lslot(l, (it & 1) ? S_DQ0 : S_DQ1);
    const int dq_cur = lslot(l, (it & 1) ? S_DQ1 : S_DQ0);
    Coefs beta = coef(H, lslot(l, S_ZQ), dq_prev, -1.0);
    Coefs mn = coef(H, lslot(l, S_SUMZ), -1, 1.0 / (double)V.n);
    Reduce R = red(H, dq_cur, lslot(l, S_DR));
    finish(H, R, launch_dir<T, T>(H, V.v, z, V.d, V.d2, V.q, V.rhs, (T*)nullptr, beta, it > 0, mn, mean, beta, R), 2);
}

template <class T>
static void update_xr(Handle* H, Lev<T>& V, T* x, int it, int l, bool first, bool skip_r, bool want)
{
    const int dq_cur = lslot(l, (it & 1) ? S_DQ1 : S_DQ0);
    Coefs alpha = coef(H, lslot(l, S_DR), dq_cur, 1.0);
    const Reduce R = red(H, lslot(l, S_RR), lslot(l, S_RSUM));
    k_update_xr<T><<<lin_grid(V.n), kBlock, 0, H->stream>>>((int)V.n, x, V.d2, V.rhs, V.q, alpha, first, skip_r, want, R,
                                                         (float*)nullptr, 1);
    check_launch();
    if (want) finish(H, R, lin_grid(V.n), 2);
}

// Whether the K-cycle at level V runs without separate x/r updates: a float32
// level with row-wave passes whose cycle starts with the plain first sweep.
template <class T>
static bool kfold_ok(const Handle* H, const Lev<T>& V, int l)
{
    if constexpr (std::is_same_v<T, float>) {
        if (!H->prm.kfold || !V.rhs2 || !rwc_geo(H, V.v).cpt) return false;
        return !(sweeps_of(H, V, l) == 1 && fused(H, sizeof(T), V.n));
    }
    return false;
}

// Direction update of K-cycle step it on residual r with the previous step's
// deferred x update (x = alpha d_old at it = 1, x += alpha d_old after).
template <class T>
static void dir_apply_fold(Handle* H, Lev<T>& V, const T* z, const T* r, int it, int l)
{
    if constexpr (std::is_same_v<T, float>) {
        const int dq_prev = lslot(l, (it & 1) ? S_DQ0 : S_DQ1);
        const int dq_cur = lslot(l, (it & 1) ? S_DQ1 : S_DQ0);
        const Coefs beta = coef(H, lslot(l, S_ZQ), dq_prev, -1.0);
        const Coefs mn = coef(H, lslot(l, S_SUMZ), -1, 1.0 / (double)V.n);
        const Coefs aprev = coef(H, lslot(l, S_DR), dq_prev, 1.0);  // read before this launch's totals
        const Reduce R = red(H, dq_cur, lslot(l, S_DR));
        const RwGeo rg = rwc_geo(H, V.v);
        with_cpt(rg, [&](auto C, auto Y) {
            constexpr int CPT = decltype(C)::value, BY = decltype(Y)::value;
            if (it == 0)
                r_dir_apply_f32<CPT, BY, false, 0><<<rg.grid, rg.block, 0, H->stream>>>(
                    V.v, z, V.d, V.d2, V.q, r, beta, mn, 0, rg.kper, rg.xcd, R, V.xk, aprev);
            else if (it == 1)
                r_dir_apply_f32<CPT, BY, true, 1><<<rg.grid, rg.block, 0, H->stream>>>(
                    V.v, z, V.d, V.d2, V.q, r, beta, mn, 0, rg.kper, rg.xcd, R, V.xk, aprev);
            else
                r_dir_apply_f32<CPT, BY, true, 2><<<rg.grid, rg.block, 0, H->stream>>>(
                    V.v, z, V.d, V.d2, V.q, r, beta, mn, 0, rg.kper, rg.xcd, R, V.xk, aprev);
        });
        check_launch();
        finish(H, R, rg.grid, 2);
    }
}

// K-cycle: kit flexible-CG steps on K_l x = rhs_l (rhs_l is used as the residual).
template <class T>
static T* kcycle(Handle* H, Hier<T>& Hh, int l)
{
    Lev<T>& V = Hh.L[l];
    const bool deepest = l + 1 >= (int)Hh.L.size() || !Hh.L[l + 1].kcyc;
    const int kit = (deepest && (long)V.n > H->prm.kbig && H->prm.kit2 > 0) ? H->prm.kit2 : H->prm.kit;
    V.d = V.d_a;
    V.d2 = V.d_b;
    if (kfold_ok(H, V, l)) {
        // the same steps without the separate x/r update launches: step it > 0's cycle forms its
        // residual r - alpha q of the previous step in its first pass (into the other residual
        // buffer), its direction update applies the previous step's x update, and the last
        // step's x update follows the loop
        const T* r = V.rhs;
        T* r_other = V.rhs2;
        for (int it = 0; it < kit; ++it) {
            T* z;
            if (it == 0) {
                z = mgcycle(H, Hh, l, r, 0, V.q);
            } else {
                const int dq_prev = lslot(l, ((it - 1) & 1) ? S_DQ1 : S_DQ0);
                const Fold<T> fd{r, V.q, r_other, coef(H, lslot(l, S_DR), dq_prev, 1.0)};
                T* rn = r_other;
                z = mgcycle(H, Hh, l, rn, 2, V.q, &fd);
                r_other = const_cast<T*>(r);
                r = rn;
            }
            dir_apply_fold(H, V, z, r, it, l);
            std::swap(V.d, V.d2);
        }
        const int dq_last = lslot(l, ((kit - 1) & 1) ? S_DQ1 : S_DQ0);
        k_update_xr<T><<<lin_grid(V.n), kBlock, 0, H->stream>>>((int)V.n, V.xk, V.d, (T*)nullptr, (const T*)nullptr,
                                                             coef(H, lslot(l, S_DR), dq_last, 1.0), kit == 1, 1, 0,
                                                             red(H, G_FN2), (float*)nullptr, 1);
        check_launch();
        return V.xk;
    }
    for (int it = 0; it < kit; ++it) {
        T* z = mgcycle(H, Hh, l, V.rhs, it > 0 ? 2 : 0, V.q);
        dir_apply(H, V, false, z, it, l, false);
        update_xr(H, V, V.xk, it, l, it == 0, it == kit - 1, false);
        std::swap(V.d, V.d2);
    }
    return V.xk;
}

// Grid of the finest-level r/q (and x) update (a grid-stride loop over element
// pairs): at most eblocks blocks (at most kMaxPartialBlocks, the partials a
// reduction can hold).  The one-element-per-step passes keep lin_grid (fewer
// blocks made them slower: the density 110 -> 187 us with 512).
static dim3 fine_grid(const Handle* H, size_t n)
{
    const size_t b = (n / 2 + kBlock - 1) / kBlock;
    return dim3((unsigned)std::max<size_t>(1, std::min<size_t>(b, (size_t)H->prm.eblocks)));
}

// One step of the finest-level flexible CG, float64 throughout (x, r, d, q and
// the operator from rho), preconditioned by one multigrid cycle in precision P:
// z = M r (the cycle also reduces sum(z), <z, q_old>, <z, r> and sum(r)),
// d = (z - mean z) + beta d_old, q = K d with <d, q>, then r -= alpha q (and the
// float32 copy of r for a float32 cycle) with ||r||^2, where
// alpha = (<z, r> - mean(z) sum(r)) / <d, q>: the numerator is <d, r> without its
// beta <d_old, r> term, which the previous step's alpha makes zero up to
// rounding, so the direction update need not read r.  (The mean term is kept:
// z may carry a large constant, and near the rounding floor mean(z) sum(r) is
// not small against <z, r>.)  The cycle's r is the float32 copy in the refined
// form.  The x update is deferred: step k applies x += alpha_{k-1} d_{k-1} while
// it reads d_{k-1} anyway, and fcg() applies the last one; the r update stores
// its alpha, by step parity, for that.
template <class P>
static void krylov_step(Handle* H, Hier<P>& Hh, int k)
{
    const pp_config& cfg = H->cfg;
    const size_t n0 = (size_t)cfg.nx * cfg.ny * cfg.nz;
    const int dq_prev = lslot(0, (k & 1) ? S_DQ0 : S_DQ1);
    const int dq_cur = lslot(0, (k & 1) ? S_DQ1 : S_DQ0);
    const int a_prev = (k & 1) ? G_ALPHA0 : G_ALPHA1;
    const int a_cur = (k & 1) ? G_ALPHA1 : G_ALPHA0;
    // the first step has no q_old: its <z, q> (unused) is taken against r instead
    H->zr_slot = lslot(0, S_DR);
    H->fsum_slot = G_FSUM;
    P* z = mgcycle<P, double>(H, Hh, 0, Hh.L[0].rhs, 4, k > 0 ? H->q64 : H->r64);
    {
        const LevelView<double> v = fine64(H);
        const Reduce R = red(H, dq_cur);
        dim3 grid;
        {
            // reads z, the float64 weights (or density) and, after the first step, d_old and x;
            // writes d, q (and x)
            TimeScope ts(H, kid<double>(KT_DIR_APPLY),
                         (double)n0 * ((double)sizeof(P) + (k > 0 ? 40.0 : 16.0) + 8.0 * weight_arrays(H, v)));
            grid = launch_dir<double, P, true>(H, v, z, H->d, H->d2, H->q64, H->r64, H->x64,
                                               coef(H, lslot(0, S_ZQ), dq_prev, -1.0), k > 0,
                                               coef(H, lslot(0, S_SUMZ), -1, 1.0 / (double)n0), 1,
                                               coef(H, a_prev, -1, 1.0), R);
        }
        finish(H, R, grid, 1);
    }
    {
        const Reduce R = red_host(H, lslot(0, S_RR), lslot(0, S_RSUM));
        Coefs alpha = coef(H, lslot(0, S_DR), dq_cur, 1.0);
        alpha.c1 = lslot(0, S_SUMZ);
        alpha.c2 = G_FSUM;
        alpha.cs = -1.0 / (double)n0;
        {
            // reads r and q; writes r and the float32 copy of r
            TimeScope ts(H, kid<double>(KT_UPDATE_XR), (double)n0 * (24.0 + (H->r32 ? 4.0 : 0.0)));
            k_update_xr<double><<<fine_grid(H, n0), kBlock, 0, H->stream>>>((int)n0, H->x64, H->d2, H->r64, H->q64,
                                                                          alpha, 0, 0, 1, R, H->r32, 0,
                                                                          H->slots + a_cur);
            check_launch();
        }
        finish(H, R, fine_grid(H, n0), 2);
    }
    std::swap(H->d, H->d2);
}

static void drop_graphs(Handle* H)
{
    for (int i = 0; i < 3; ++i) {
        if (H->kexec[i]) {
            (void)hipGraphExecDestroy(H->kexec[i]);
            H->kexec[i] = nullptr;
        }
    }
}

// Flexible CG on the finest level until ||r|| <= rnorm_stop or max_it steps;
// r64 (and r32) must hold the residual of x64.  Returns the steps taken.
// Steps are replayed from captured graphs when possible: every pointer and
// slot a step uses is fixed by the parity of its index.
template <class P>
static int fcg(Handle* H, Hier<P>& Hh, double rnorm_stop, int max_it, double* rnorm_out)
{
    H->d = H->d_a;
    H->d2 = H->d_b;
    int k = 0;
    double rn = -1.0;
    for (; k < max_it; ++k) {
        const int kind = k == 0 ? 0 : ((k & 1) ? 1 : 2);
        // kernel timing brackets every launch with events, which graphs cannot carry:
        // timed steps are launched directly
        const bool graphs = H->use_graphs && !H->timing;
        if (graphs && !H->kexec[kind]) {
            double* d0 = H->d;
            double* d1 = H->d2;
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamBeginCapture(H->stream, hipStreamCaptureModeRelaxed);
            if (e == hipSuccess) {
                try {
                    krylov_step(H, Hh, k);
                } catch (...) {
                    (void)hipStreamEndCapture(H->stream, &g);
                    if (g) (void)hipGraphDestroy(g);
                    throw;
                }
                e = hipStreamEndCapture(H->stream, &g);
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&H->kexec[kind], g, nullptr, nullptr, 0);
            if (g) (void)hipGraphDestroy(g);
            H->d = d0;  // capture ran nothing: restore and replay below
            H->d2 = d1;
            if (e != hipSuccess) {  // capture unavailable: launch directly from now on
                (void)hipGetLastError();
                H->kexec[kind] = nullptr;
                H->use_graphs = false;
            }
        }
        const bool replay = graphs && H->use_graphs && H->kexec[kind];
        if (replay) {
            PP_HIP(hipGraphLaunch(H->kexec[kind], H->stream));
            std::swap(H->d, H->d2);
        } else {
            krylov_step(H, Hh, k);
        }
        fetch_slots(H, lslot(0, S_RR), 1);
        rn = std::sqrt(std::max(0.0, H->host_slots[lslot(0, S_RR)]));
        if (!(rn == rn)) throw Fail(PP_ERR_NONFINITE, "non-finite residual during the iteration");
        if (rn <= rnorm_stop) { ++k; break; }
    }
    if (k > 0) {  // the deferred x += alpha d of the last step
        const size_t n0 = (size_t)H->cfg.nx * H->cfg.ny * H->cfg.nz;
        const int last = k - 1;
        const Coefs a = coef(H, (last & 1) ? G_ALPHA1 : G_ALPHA0, -1, 1.0);
        k_update_xr<double><<<fine_grid(H, n0), kBlock, 0, H->stream>>>((int)n0, H->x64, H->d, H->r64, H->q64, a, 0, 1, 0,
                                                                    red(H, G_FN2), (float*)nullptr, 1);
        check_launch();
    }
    if (rnorm_out) *rnorm_out = rn;
    return k;
}

// ---------------------------------------------------------------- set-up

static void set_density(Handle* H, const double* rho)
{
    const pp_config& cfg = H->cfg;
    const int nl = H->nlev;
    const size_t n0 = (size_t)cfg.nx * cfg.ny * cfg.nz;
    PP_HIP(hipEventRecord(H->ev0, H->stream));
    const bool fine_rho = weights_from_density(H->prm);
    auto bad_density = [&]() {
        return Fail(PP_ERR_NONFINITE, "density has " + std::to_string((long long)H->host_slots[G_RHOBAD]) +
                                          " entries that are not finite or not > 0");
    };
    // one pass over the density for the finest level and the first coarse one (the validation's
    // count is checked at the end; the handle holds no density until then)
    const bool one_pass = fine_rho && nl >= 2 && H->prm.onepass;
    if (one_pass) {
        const Geo g = geo(H->lnx[1], H->lny[1], H->lnz[1]);
        const Reduce R = red(H, G_RHOBAD);
        if (H->c64[0].invd)
            k_fine_setup<true><<<g.grid, g.block, 0, H->stream>>>(cfg.nx, cfg.ny, cfg.nz, rho, H->rho64, H->rho32,
                                                                  H->c64[0].invd, H->c32[0].invd, H->c64[1].wx,
                                                                  H->c64[1].wy, H->c64[1].wz, g.kper, R);
        else
            k_fine_setup<false><<<g.grid, g.block, 0, H->stream>>>(cfg.nx, cfg.ny, cfg.nz, rho, H->rho64, H->rho32,
                                                                   nullptr, H->c32[0].invd, H->c64[1].wx, H->c64[1].wy,
                                                                   H->c64[1].wz, g.kper, R);
        check_launch();
        finish(H, red_host(H, G_RHOBAD), g.grid, 1);
    } else {
        // validate: finite and > 0
        k_sum_check<<<lin_grid(n0), kBlock, 0, H->stream>>>((int)n0, rho, 1, red(H, G_RHOSUM, G_RHOBAD));
        check_launch();
        finish(H, red_host(H, G_RHOSUM, G_RHOBAD), lin_grid(n0), 2);
        fetch_slots(H, G_RHOSUM, 2);
        if (H->host_slots[G_RHOBAD] != 0.0) throw bad_density();
        // the handle's own copies of the density (the caller keeps rho)
        k_take_density<<<lin_grid(n0), kBlock, 0, H->stream>>>((int)n0, rho, H->rho64, H->rho32);
        check_launch();
    }
    for (int l = 0; l < nl; ++l) {
        Geo g = geo(H->lnx[l], H->lny[l], H->lnz[l]);
        if (one_pass && l == 0) continue;
        if (l == 0 && fine_rho) {
            // no stored finest weights: 1/D from the density (float64 for the float64 cycle, float32
            // as the float32 passes form their weights for the float32 cycle)
            if (H->c64[0].invd)
                k_fine_diag<<<g.grid, g.block, 0, H->stream>>>(cfg.nx, cfg.ny, cfg.nz, H->rho64, H->c64[0].invd,
                                                               H->c32[0].invd, g.kper);
            else
                k_fine_diag32<<<g.grid, g.block, 0, H->stream>>>(cfg.nx, cfg.ny, cfg.nz, H->rho32, H->c32[0].invd,
                                                                 g.kper);
            check_launch();
            continue;
        }
        if (l == 0)
            k_fine_faces<<<g.grid, g.block, 0, H->stream>>>(cfg.nx, cfg.ny, cfg.nz, rho, H->c64[0].wx, H->c64[0].wy,
                                                            H->c64[0].wz, g.kper);
        else if (l == 1 && one_pass) {
            // formed by k_fine_setup
        }
        else if (l == 1 && fine_rho)
            k_coarsen_rho<<<g.grid, g.block, 0, H->stream>>>(cfg.nx, cfg.ny, cfg.nz, H->rho64, H->lnx[1], H->lny[1],
                                                             H->lnz[1], H->c64[1].wx, H->c64[1].wy, H->c64[1].wz, g.kper);
        else
            k_coarsen<<<g.grid, g.block, 0, H->stream>>>(H->lnx[l - 1], H->lny[l - 1], H->lnz[l - 1], H->c64[l - 1].wx,
                                                         H->c64[l - 1].wy, H->c64[l - 1].wz, H->lnx[l], H->lny[l], H->lnz[l],
                                                         H->c64[l].wx, H->c64[l].wy, H->c64[l].wz, g.kper);
        check_launch();
        k_level_finish<<<g.grid, g.block, 0, H->stream>>>(H->lnx[l], H->lny[l], H->lnz[l], H->c64[l].wx, H->c64[l].wy,
                                                          H->c64[l].wz, H->c64[l].invd, H->c32[l].wx, H->c32[l].wy,
                                                          H->c32[l].wz, H->c32[l].invd, H->c32[l].hx, H->c32[l].hy,
                                                          H->c32[l].hz, g.kper);
        check_launch();
    }
    if (H->M64) {
        // after the coarsest weights (and every use of the previous inverse: the same stream) on
        // the second stream; the next solve waits for it before its first cycle.  A set-up that
        // follows before any solve may rewrite the weights a previous inverse is still reading;
        // that inverse's result is then overwritten by this one, queued after it on the same
        // stream, and nothing reads the matrix in between
        const int l = nl - 1;
        PP_HIP(hipEventRecord(H->ev_coarse, H->stream));
        PP_HIP(hipStreamWaitEvent(H->side, H->ev_coarse, 0));
        k_dense_inverse<<<1, kDenseThreads, 0, H->side>>>(H->lnx[l], H->lny[l], H->lnz[l], H->c64[l].wx,
                                                          H->c64[l].wy, H->c64[l].wz, H->M64, H->M32);
        check_launch();
        PP_HIP(hipEventRecord(H->ev_dense, H->side));
        H->dense_pending = true;
    }
    PP_HIP(hipEventRecord(H->ev1, H->stream));
    PP_HIP(hipEventSynchronize(H->ev1));
    if (one_pass) {
        fetch_slots(H, G_RHOBAD, 1);
        if (H->host_slots[G_RHOBAD] != 0.0) throw bad_density();
    }
    float ms = 0.f;
    PP_HIP(hipEventElapsedTime(&ms, H->ev0, H->ev1));
    H->setup_ms = ms;
    H->have_density = true;
}

// f = -h^2 (b - mean b); returns ||f||.
static double prepare_rhs(Handle* H, const double* rhs)
{
    const pp_config& cfg = H->cfg;
    const size_t n0 = (size_t)cfg.nx * cfg.ny * cfg.nz;
    k_sum_check<<<lin_grid(n0), kBlock, 0, H->stream>>>((int)n0, rhs, 0, red(H, G_BSUM, G_BBAD));
    check_launch();
    finish(H, red_host(H, G_BSUM, G_BBAD), lin_grid(n0), 2);
    // the shift reads the mean from the device slot; the count of non-finite entries is checked
    // with ||f|| after it (one wait for the host instead of two)
    k_shift_scale<<<lin_grid(n0), kBlock, 0, H->stream>>>((int)n0, rhs, H->f64, -cfg.h * cfg.h, coef(H, G_BSUM, -1, 1.0 / (double)n0),
                                                          1, red(H, G_FN2));
    check_launch();
    finish(H, red_host(H, G_FN2), lin_grid(n0), 1);
    fetch_slots(H, G_BSUM, G_FN2 - G_BSUM + 1);
    if (H->host_slots[G_BBAD] != 0.0)
        throw Fail(PP_ERR_NONFINITE, "rhs has " + std::to_string((long long)H->host_slots[G_BBAD]) + " non-finite entries");
    return std::sqrt(H->host_slots[G_FN2]);
}

// r64 = f64 - K x in float64; returns ||r|| (sum(r) in slot G_TRSUM, sum(x) in
// G_XSUM).  xc (or null) receives a copy of x, r32 (or null) the float32 copy of r.
static double true_residual(Handle* H, const double* x, double* xc, float* r32)
{
    const pp_config& cfg = H->cfg;
    const LevelView<double> v = fine64(H);
    dim3 grid;
    {
        // reads f, x and the float64 weights (or density); writes r (and the copies)
        TimeScope ts(H, kid<double>(KT_TRUE_RESIDUAL),
                     (double)cfg.nx * cfg.ny * cfg.nz *
                         (24.0 + 8.0 * weight_arrays(H, v) + (xc ? 8.0 : 0.0) + (r32 ? 4.0 : 0.0)));
        const Reduce R = red(H, G_TRR, G_TRSUM, G_XSUM);
        const RwGeo rg = rw_geo(H, v);
        if (rg.cpt) {
            with_cpt_rw(rg, [&](auto C, auto Y, auto P) {
                r_true_residual<decltype(C)::value, decltype(Y)::value, decltype(P)::value>
                    <<<rg.grid, rg.block, 0, H->stream>>>(v, H->f64, x, H->r64, rg.kper, rg.xcd, R, xc, r32);
            });
            grid = rg.grid;
        } else if (H->prm.march) {
            const MGeo g = march_geo(H, v, H->prm.mbx);
            with_bx(g.bx, [&](auto B) {
                with_rho(v, [&](auto W) {
                    m_true_residual<decltype(B)::value, decltype(W)::value>
                        <<<g.grid, g.block, 0, H->stream>>>(v, H->f64, x, H->r64, g.kper, xcd_of(H, v), R, xc, r32);
                });
            });
            grid = g.grid;
        } else {
            const Geo g = geo(cfg.nx, cfg.ny, cfg.nz);
            k_true_residual<<<g.grid, g.block, 0, H->stream>>>(v, H->f64, x, H->r64, g.kper, R, xc, r32);
            grid = g.grid;
        }
        check_launch();
    }
    finish(H, red_host(H, G_TRR, G_TRSUM, G_XSUM), grid, 3);
    fetch_slots(H, G_TRR, 2);
    return std::sqrt(std::max(0.0, H->host_slots[G_TRR]));
}

// out = x - mean(x), with sum(x) already in slot G_XSUM (the last true_residual of x)
static void remove_mean(Handle* H, const double* x, double* out)
{
    const size_t n0 = (size_t)H->cfg.nx * H->cfg.ny * H->cfg.nz;
    k_shift_scale<<<lin_grid(n0), kBlock, 0, H->stream>>>((int)n0, x, out, 1.0, coef(H, G_XSUM, -1, 1.0 / (double)n0), 0,
                                                          red(H, G_FN2));
    check_launch();
}

static int solve(Handle* H, const double* rhs, double* p, pp_stats* st)
{
    auto t0 = std::chrono::steady_clock::now();
    const pp_config& cfg = H->cfg;
    const size_t n0 = (size_t)cfg.nx * cfg.ny * cfg.nz;
    const int max_it = cfg.max_iters > 0 ? cfg.max_iters : 1000;
    const double fn = prepare_rhs(H, rhs);
    int iters = 0, restarts = 0;
    double rel = 0.0;
    bool converged = true;
    if (fn == 0.0) {
        PP_HIP(hipMemsetAsync(p, 0, sizeof(double) * n0, H->stream));
        PP_HIP(hipStreamSynchronize(H->stream));
    } else {
        converged = false;
        bool first = true;
        for (;;) {
            // r64 = f - K x (and its float32 copy for a float32 cycle); the first one reads the
            // caller's guess and leaves the handle's copy of it in x64
            const double rn = first ? true_residual(H, p, H->x64, H->r32) : true_residual(H, H->x64, nullptr, H->r32);
            first = false;
            rel = rn / fn;
            if (rel <= cfg.tol) { converged = true; break; }
            if (!(rel == rel)) throw Fail(PP_ERR_NONFINITE, "non-finite residual during the iteration");
            if (iters >= max_it || restarts >= 50) break;
            if (H->dense_pending) {  // the coarsest inverse of the last set-up (second stream)
                PP_HIP(hipStreamWaitEvent(H->stream, H->ev_dense, 0));
                H->dense_pending = false;
            }
            if (H->prm.mg_solver) {
                // the paper's form: multigrid cycles with red-black SOR as the solver, x += M (f - K x)
                double* z = mgcycle<double, double>(H, H->h64, 0, H->r64, 0, nullptr);
                k_update_xr<double><<<fine_grid(H, n0), kBlock, 0, H->stream>>>((int)n0, H->x64, z, H->r64, H->q64,
                                                                            coef(H, G_ONE, -1, 1.0), 0, 1, 0,
                                                                            red(H, G_FN2), (float*)nullptr, 1);
                check_launch();
                ++iters;
                continue;
            }
            if (cfg.mode == PP_FP64) iters += fcg(H, H->h64, cfg.tol * fn, max_it - iters, nullptr);
            else iters += fcg(H, H->h32, cfg.tol * fn, max_it - iters, nullptr);
            ++restarts;  // the recursion's residual met the tolerance: check the true one
        }
        // every exit from the loop follows a true residual of x: p = x - mean(x) with its sum of
        // x, and that residual is p's (K 1 = 0: the shift changes it only by rounding)
        remove_mean(H, H->x64, p);
    }
    PP_HIP(hipStreamSynchronize(H->stream));
    auto t1 = std::chrono::steady_clock::now();
    if (H->timing) collect_timing(H);
    if (st) {
        st->iters = iters;
        st->outer_iters = restarts;
        st->inner_iters_total = cfg.mode == PP_FP64 ? 0 : iters;
        st->rel_residual = rel;
        st->setup_ms = H->setup_ms;
        st->solve_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
        st->device_bytes = H->arena_bytes;
    }
    if (!converged) throw Fail(PP_ERR_NOT_CONVERGED, "not converged: relative residual " + std::to_string(rel));
    return PP_OK;
}

static void read_env(Params& p, const pp_config* cfg = nullptr)
{
    if (cfg && cfg->pre_sweeps > 0) p.nu0 = cfg->pre_sweeps;
    if (cfg && cfg->post_sweeps > 0) p.nuc = cfg->post_sweeps;
    if (cfg && cfg->omega > 0.0) p.omega = cfg->omega;
    if (cfg && (cfg->flags & PP_FLAG_MG_SOLVER)) {
        p.mg_solver = true;
        p.kmax = 0;  // plain V-cycles: no Krylov steps anywhere in this form
        p.nuv = 0;   // and post_sweeps (default 2) on every coarse level: as a stationary
                     // iteration the cycle needs them (with one sweep it diverges)
        if (cfg->flags & PP_FLAG_W_CYCLE) p.gamma = 2;  // two visits of each coarse level
    }
    if (const char* s = getenv("PP_KMAX")) p.kmax = atoi(s);
    if (const char* s = getenv("PP_KMIN")) p.kmin = std::max(0, atoi(s));
    if (const char* s = getenv("PP_KIT")) p.kit = std::max(1, atoi(s));
    if (const char* s = getenv("PP_WC")) p.wc = atof(s);
    if (const char* s = getenv("PP_NU0")) p.nu0 = std::max(1, atoi(s));
    if (const char* s = getenv("PP_NUC")) p.nuc = std::max(1, atoi(s));
    if (const char* s = getenv("PP_GRAPHS")) p.graphs = atoi(s) != 0;
    if (const char* s = getenv("PP_HW")) p.hw = atoi(s) != 0;
    if (const char* s = getenv("PP_HWMIN")) p.hwmin = std::max(0L, atol(s));
    if (const char* s = getenv("PP_FUSE")) p.fuse = std::max(0, std::min(2, atoi(s)));
    if (const char* s = getenv("PP_PFUSE")) p.pfuse = atoi(s) != 0;
    if (const char* s = getenv("PP_FBIG")) p.fbig = std::max(0L, atol(s));
    if (const char* s = getenv("PP_FSMALL")) p.fsmall = std::max(0L, atol(s));
    if (const char* s = getenv("PP_OBLOCKS")) p.oblocks = std::max(8, std::min(1 << 16, atoi(s)));
    if (const char* s = getenv("PP_TAIL")) p.tail = atoi(s) != 0;
    if (const char* s = getenv("PP_TAILMAX")) p.tail_max = std::max(2, std::min(kTailMaxCells, atoi(s)));
    if (const char* s = getenv("PP_OMEGA")) p.omega = atof(s);
    if (const char* s = getenv("PP_KIT2")) p.kit2 = std::max(0, atoi(s));
    if (const char* s = getenv("PP_KBIG")) p.kbig = std::max(0L, atol(s));
    if (const char* s = getenv("PP_NUV")) p.nuv = std::max(0, atoi(s));
    if (const char* s = getenv("PP_NU1")) p.nu1 = std::max(0, atoi(s));
    if (const char* s = getenv("PP_NUK2")) p.nuk2 = std::max(0, atoi(s));
    if (const char* s = getenv("PP_MARCH")) p.march = atoi(s) != 0;
    if (const char* s = getenv("PP_XCD")) p.xcd = atoi(s);
    if (const char* s = getenv("PP_OXCD")) p.oxcd = atoi(s);
    if (const char* s = getenv("PP_RHO")) p.rho = atoi(s) != 0;
    if (const char* s = getenv("PP_FBLOCKS")) p.fblocks = std::max(32, std::min(kMaxRedBlocks, atoi(s)));
    if (const char* s = getenv("PP_MBLOCKS")) p.mblocks = std::max(64, std::min(kMaxRedBlocks, atoi(s)));
    if (const char* s = getenv("PP_RW")) p.rw = atoi(s) != 0;
    if (const char* s = getenv("PP_RWDIR")) p.rwdir = std::max(0, std::min(2, atoi(s)));
    if (const char* s = getenv("PP_RWBLOCKS")) p.rwblocks = std::max(8, std::min(kMaxPartialBlocks, atoi(s)));
    if (const char* s = getenv("PP_RWXCD")) p.rwxcd = atoi(s) != 0;
    if (const char* s = getenv("PP_RWROWS")) p.rwrows = atoi(s) <= 4 ? 4 : 8;
    if (const char* s = getenv("PP_RWSPLIT")) p.rwsplit = atoi(s) == 2 ? 2 : 1;
    if (const char* s = getenv("PP_RWSROWS")) p.rwsrows = atoi(s) <= 4 ? 4 : (atoi(s) <= 6 ? 6 : 8);
    if (const char* s = getenv("PP_RWSBLOCKS")) p.rwsblocks = std::max(8, std::min(kMaxPartialBlocks, atoi(s)));
    if (const char* s = getenv("PP_RWSXCD")) p.rwsxcd = atoi(s) != 0;
    if (const char* s = getenv("PP_RWCROWS")) p.rwcrows = atoi(s) <= 4 ? 4 : 8;
    if (const char* s = getenv("PP_EBLOCKS")) p.eblocks = std::max(64, std::min(kMaxPartialBlocks, atoi(s)));
    if (const char* s = getenv("PP_KFOLD")) p.kfold = atoi(s) != 0;
    if (const char* s = getenv("PP_ONEPASS")) p.onepass = atoi(s) != 0;
    if (const char* s = getenv("PP_RWCBLOCKS")) p.rwcblocks = std::max(8, std::min(kMaxPartialBlocks, atoi(s)));
    if (const char* s = getenv("PP_RWCXCD")) p.rwcxcd = atoi(s) != 0;
    if (const char* s = getenv("PP_RWF")) p.rwf = atoi(s) != 0;
    if (const char* s = getenv("PP_RWC")) p.rwc = atoi(s) != 0;
    if (const char* s = getenv("PP_RWFXCD")) p.rwfxcd = atoi(s) != 0;
    if (const char* s = getenv("PP_RWFROWS")) p.rwfrows = atoi(s) >= 16 ? 16 : (atoi(s) >= 12 ? 12 : 8);
    if (const char* s = getenv("PP_RWFBLOCKS")) p.rwfblocks = std::max(8, std::min(kMaxPartialBlocks, atoi(s)));
    if (const char* s = getenv("PP_MBX")) {
        const int b = atoi(s);
        p.mbx = (b >= 64) ? 64 : (b >= 32) ? 32 : (b >= 16) ? 16 : 8;
    }
}

}  // namespace pp

// ---------------------------------------------------------------- C ABI

using namespace pp;

struct pp_handle_s {
    Handle h;
};

template <class F>
static int guarded(pp_handle h, F&& f)
{
    try {
        return f();
    } catch (const Fail& e) {
        if (h) h->h.err = e.msg;
        else g_thread_err = e.msg;
        return e.code;
    } catch (const std::exception& e) {
        if (h) h->h.err = e.what();
        else g_thread_err = e.what();
        return PP_ERR_HIP;
    }
}

// Relative residual ||bbar - A p|| / ||bbar|| of step 11 on the device:
// density check, sum of b, then the two squared norms by the plane-marching
// operator, each reduction through `partials` (kMaxPartialBlocks * kMaxRed
// doubles) into `slots` (8 doubles).  Synchronises `st`.
enum : int { R_RHOSUM = 0, R_RHOBAD, R_BSUM, R_BBAD, R_RR, R_BB, kRelSlots = 8 };
static int rel_residual_on(hipStream_t st, int nx, int ny, int nz, double h, const double* rho, const double* rhs,
                           const double* p, double* rel_out, double* partials, double* slots)
{
    const size_t n = (size_t)nx * ny * nz;
    auto R = [&](int a, int b) {
        Reduce r;
        r.partials = partials;
        r.out = slots;
        r.slot[0] = a; r.slot[1] = b; r.slot[2] = 0; r.slot[3] = 0;
        return r;
    };
    const dim3 lg = lin_grid(n);
    k_sum_check<<<lg, kBlock, 0, st>>>((int)n, rho, 1, R(R_RHOSUM, R_RHOBAD));
    check_launch();
    k_reduce_finish<<<1, kBlock, 0, st>>>(R(R_RHOSUM, R_RHOBAD), (int)(lg.x * lg.y * lg.z), 2);
    check_launch();
    k_sum_check<<<lg, kBlock, 0, st>>>((int)n, rhs, 0, R(R_BSUM, R_BBAD));
    check_launch();
    k_reduce_finish<<<1, kBlock, 0, st>>>(R(R_BSUM, R_BBAD), (int)(lg.x * lg.y * lg.z), 2);
    check_launch();
    const MGeo g = mgeo(nx, ny, nz, 64, false, 512, kMarchThreads<double, true>);
    const LevelView<double> v{nx, ny, nz, nullptr, nullptr, nullptr, nullptr, rho};
    with_bx(g.bx, [&](auto B) {
        m_rel_residual<decltype(B)::value><<<g.grid, g.block, 0, st>>>(v, p, rhs, 1.0 / (h * h),
                                                                       Coefs{slots, R_BSUM, -1, 1.0 / (double)n}, g.kper,
                                                                       R(R_RR, R_BB));
    });
    check_launch();
    k_reduce_finish<<<1, kBlock, 0, st>>>(R(R_RR, R_BB), (int)(g.grid.x * g.grid.y * g.grid.z), 2);
    check_launch();
    double host[kRelSlots];
    PP_HIP(hipMemcpyAsync(host, slots, sizeof(host), hipMemcpyDeviceToHost, st));
    PP_HIP(hipStreamSynchronize(st));
    if (host[R_RHOBAD] != 0.0) throw Fail(PP_ERR_NONFINITE, "density not finite or not > 0");
    if (host[R_BBAD] != 0.0) throw Fail(PP_ERR_NONFINITE, "rhs not finite");
    const double rr = std::sqrt(host[R_RR]), bb = std::sqrt(host[R_BB]);
    *rel_out = bb > 0.0 ? rr / bb : (rr > 0.0 ? HUGE_VAL : 0.0);
    return PP_OK;
}

// Checks of the residual entry points: sizes, pointers, and a launch whose
// partial sums fit the kMaxPartialBlocks partials.
static int rel_residual_args(int nx, int ny, int nz, double h, const void* rho, const void* rhs, const void* p,
                             const void* rel_out)
{
    if (!rho || !rhs || !p || !rel_out) { g_thread_err = "null pointer"; return PP_ERR_INVALID; }
    if (nx < 1 || ny < 1 || nz < 1 || !(h > 0.0) || !std::isfinite(h)) { g_thread_err = "bad sizes or h"; return PP_ERR_INVALID; }
    if ((size_t)nx * ny * nz + (size_t)nx * ny > (size_t)INT_MAX) {
        g_thread_err = "grid too large (32-bit cell indices)";
        return PP_ERR_INVALID;
    }
    const MGeo g = mgeo(nx, ny, nz, 64, false, 512, kMarchThreads<double, true>);
    if ((size_t)g.grid.x * g.grid.y * g.grid.z > (size_t)kMaxPartialBlocks) {
        g_thread_err = "cross-section too large: more than 4096 tiles of 64 x 8 cells per plane";
        return PP_ERR_INVALID;
    }
    return PP_OK;
}

// Scratch of pp_rel_residual_noalloc: the partial sums and result slots of its
// reductions (131136 bytes).  Every GPU the library runs on holds its own copy
// until the process ends, and every call on that GPU shares it.  Host code uses
// the per-device address from hipGetSymbolAddress, never this name.
static __device__ __align__(256) double scratch[(size_t)kMaxPartialBlocks * kMaxRed + kRelSlots];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
static double* scratch_of_current_device()
{
    int dev = -1;
    PP_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) throw Fail(PP_ERR_INVALID, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            throw Fail(PP_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = static_cast<double*>(ptr);
    }
    return g_scratch_ptr[dev];
}

// Handle-less stencil entry points index cells with 32-bit ints.
static bool grid_fits_int(int nx, int ny, int nz)
{
    return (size_t)nx * ny * nz + (size_t)nx * ny <= (size_t)INT_MAX;
}

extern "C" {

const char* pp_version(void) { return "ppsolve 0.1 (gfx950)"; }

size_t pp_footprint_bytes(const pp_config* cfg)
{
    if (!valid_cfg(cfg, nullptr)) return 0;
    Handle tmp;
    read_env(tmp.prm, cfg);
    return plan(&tmp, *cfg, nullptr);
}

int pp_create(const pp_config* cfg, void* hip_stream, pp_handle* out)
{
    if (out) *out = nullptr;
    std::string why;
    if (!out) { g_thread_err = "out is null"; return PP_ERR_INVALID; }
    if (!valid_cfg(cfg, &why)) { g_thread_err = why; return PP_ERR_INVALID; }
    pp_handle h = new (std::nothrow) pp_handle_s;
    if (!h) { g_thread_err = "host allocation failed"; return PP_ERR_OOM; }
    Handle* H = &h->h;
    H->cfg = *cfg;
    H->user = (hipStream_t)hip_stream;
    read_env(H->prm, cfg);
    H->use_graphs = H->prm.graphs;
    int rc = guarded(nullptr, [&]() -> int {
        PP_HIP(hipGetDevice(&H->device));
        size_t bytes = plan(H, *cfg, nullptr);
        if (const char* s = getenv("PP_FAULT_OOM_AT")) {
            if ((size_t)atoll(s) <= bytes) throw Fail(PP_ERR_OOM, "injected allocation failure");
        }
        hipError_t e = hipMalloc((void**)&H->arena, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            H->arena = nullptr;
            throw Fail(PP_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
        }
        H->arena_bytes = bytes;
        plan(H, *cfg, H->arena);
        PP_HIP(hipStreamCreateWithFlags(&H->stream, hipStreamNonBlocking));
        PP_HIP(hipEventCreateWithFlags(&H->ev_in, hipEventDisableTiming));
        PP_HIP(hipEventCreateWithFlags(&H->ev_out, hipEventDisableTiming));
        PP_HIP(hipHostMalloc((void**)&H->host_slots, sizeof(double) * kSlots, hipHostMallocMapped | hipHostMallocCoherent));
        {
            // device view of the host slots: reductions the host reads write their totals there
            void* dv = nullptr;
            if (getenv("PP_HOSTSLOTS") && atoi(getenv("PP_HOSTSLOTS")) == 0) dv = nullptr;
            else if (hipHostGetDevicePointer(&dv, H->host_slots, 0) != hipSuccess) {
                (void)hipGetLastError();
                dv = nullptr;
            }
            H->host_slots_dev = static_cast<double*>(dv);
        }
        PP_HIP(hipEventCreate(&H->ev0));
        PP_HIP(hipEventCreate(&H->ev1));
        PP_HIP(hipStreamCreateWithFlags(&H->side, hipStreamNonBlocking));
        PP_HIP(hipEventCreateWithFlags(&H->ev_coarse, hipEventDisableTiming));
        PP_HIP(hipEventCreateWithFlags(&H->ev_dense, hipEventDisableTiming));
        PP_HIP(hipMemsetAsync(H->slots, 0, kSlots * sizeof(double), H->stream));
        {
            double one = 1.0;
            write_slots(H, G_ONE, &one, 1);
        }
        PP_HIP(hipStreamSynchronize(H->stream));
        return PP_OK;
    });
    if (rc != PP_OK) {
        if (H->stream) (void)hipStreamDestroy(H->stream);
        if (H->ev_in) (void)hipEventDestroy(H->ev_in);
        if (H->ev_out) (void)hipEventDestroy(H->ev_out);
        if (H->arena) (void)hipFree(H->arena);
        if (H->host_slots) (void)hipHostFree(H->host_slots);
        if (H->ev0) (void)hipEventDestroy(H->ev0);
        if (H->ev1) (void)hipEventDestroy(H->ev1);
        if (H->side) (void)hipStreamDestroy(H->side);
        if (H->ev_coarse) (void)hipEventDestroy(H->ev_coarse);
        if (H->ev_dense) (void)hipEventDestroy(H->ev_dense);
        delete h;
        return rc;
    }
    *out = h;
    return PP_OK;
}

int pp_set_density(pp_handle h, const double* rho)
{
    if (!h) { g_thread_err = "null handle"; return PP_ERR_INVALID; }
    if (!rho) { h->h.err = "rho is null"; return PP_ERR_INVALID; }
    return guarded(h, [&]() -> int {
        PP_HIP(hipSetDevice(h->h.device));
        h->h.have_density = false;
        enter(&h->h);
        set_density(&h->h, rho);
        leave(&h->h);
        return PP_OK;
    });
}

int pp_solve(pp_handle h, const double* rhs, double* p, pp_stats* st)
{
    if (!h) { g_thread_err = "null handle"; return PP_ERR_INVALID; }
    if (!rhs || !p) { h->h.err = "rhs or p is null"; return PP_ERR_INVALID; }
    if (!h->h.have_density) { h->h.err = "pp_solve before pp_set_density"; return PP_ERR_STATE; }
    return guarded(h, [&]() -> int {
        PP_HIP(hipSetDevice(h->h.device));
        enter(&h->h);
        int rc = PP_OK;
        try {
            rc = solve(&h->h, rhs, p, st);
        } catch (...) {
            (void)hipStreamSynchronize(h->h.stream);
            leave(&h->h);
            throw;
        }
        leave(&h->h);
        return rc;
    });
}

int pp_apply(pp_handle h, const double* x, double* y)
{
    if (!h) { g_thread_err = "null handle"; return PP_ERR_INVALID; }
    if (!x || !y) { h->h.err = "x or y is null"; return PP_ERR_INVALID; }
    if (!h->h.have_density) { h->h.err = "pp_apply before pp_set_density"; return PP_ERR_STATE; }
    return guarded(h, [&]() -> int {
        Handle* H = &h->h;
        PP_HIP(hipSetDevice(H->device));
        enter(H);
        const double inv_h2 = 1.0 / (H->cfg.h * H->cfg.h);
        const RwGeo rg = rw_geo(H, fine64(H));
        if (rg.cpt) {
            // the finest-level operator exactly as the solve's passes form it
            const LevelView<double> v = fine64(H);
            with_cpt_rw(rg, [&](auto C, auto Y, auto P) {
                r_apply<decltype(C)::value, decltype(Y)::value, decltype(P)::value>
                    <<<rg.grid, rg.block, 0, H->stream>>>(v, x, y, inv_h2, rg.kper, rg.xcd);
            });
        } else if (H->prm.march) {
            const LevelView<double> v = fine64(H);
            const MGeo g = march_geo(H, v, H->prm.mbx);
            with_bx(g.bx, [&](auto B) {
                with_rho(v, [&](auto W) {
                    m_apply<decltype(B)::value, decltype(W)::value>
                        <<<g.grid, g.block, 0, H->stream>>>(v, x, y, inv_h2, g.kper, xcd_of(H, v));
                });
            });
        } else {
            Geo g = geo(H->cfg.nx, H->cfg.ny, H->cfg.nz);
            const LevelView<double> v{H->cfg.nx, H->cfg.ny, H->cfg.nz, H->c64[0].wx, H->c64[0].wy, H->c64[0].wz, nullptr};
            k_apply_a<<<g.grid, g.block, 0, H->stream>>>(v, inv_h2, x, y, g.kper);
        }
        check_launch();
        leave(H);
        PP_HIP(hipStreamSynchronize(H->stream));
        return PP_OK;
    });
}

// Common checks of the cycle-leg entry points; the finest level must coarsen.
static int leg_checks(pp_handle h, bool ok_ptrs)
{
    if (!h) { g_thread_err = "null handle"; return PP_ERR_INVALID; }
    if (!ok_ptrs) { h->h.err = "null array"; return PP_ERR_INVALID; }
    if (!h->h.have_density) { h->h.err = "cycle pass before pp_set_density"; return PP_ERR_STATE; }
    if (h->h.nlev < 2) { h->h.err = "the grid does not coarsen (nx, ny even, nz divisible by 4, more than 64 cells)"; return PP_ERR_INVALID; }
    return PP_OK;
}

int pp_presmooth_restrict(pp_handle h, const void* f, void* x, void* rc)
{
    if (int e = leg_checks(h, f && x && rc)) return e;
    return guarded(h, [&]() -> int {
        Handle* H = &h->h;
        PP_HIP(hipSetDevice(H->device));
        enter(H);
        if (H->cfg.mode == PP_FP64) {
            Lev<double>& V = H->h64.L[0];
            cycle_pre<double>(H, V, 0, sweeps_of(H, V, 0), (const double*)f, (double*)x, (double*)rc);
        } else {
            Lev<float>& V = H->h32.L[0];
            cycle_pre<float>(H, V, 0, sweeps_of(H, V, 0), (const float*)f, (float*)x, (float*)rc);
        }
        leave(H);
        PP_HIP(hipStreamSynchronize(H->stream));
        return PP_OK;
    });
}

int pp_prolong_postsmooth(pp_handle h, const void* f, const void* x, const void* e, double wc, void* z, const double* q,
                          double* dots)
{
    if (int st = leg_checks(h, f && x && e && z && (!q || dots))) return st;
    return guarded(h, [&]() -> int {
        Handle* H = &h->h;
        PP_HIP(hipSetDevice(H->device));
        enter(H);
        const int ndot = q ? 2 : 0;
        if (H->cfg.mode == PP_FP64) {
            Lev<double>& V = H->h64.L[0];
            cycle_post<double, double>(H, V, 0, sweeps_of(H, V, 0), (const double*)f, (const double*)x, (const double*)e,
                                       wc, (double*)z, ndot, q);
        } else {
            Lev<float>& V = H->h32.L[0];
            cycle_post<float, double>(H, V, 0, sweeps_of(H, V, 0), (const float*)f, (const float*)x, (const float*)e,
                                      (float)wc, (float*)z, ndot, q);
        }
        leave(H);
        if (q) {
            read_slots(H, lslot(0, 0), kLevSlots);
            dots[0] = H->host_slots[lslot(0, S_SUMZ)];
            dots[1] = H->host_slots[lslot(0, S_ZQ)];
        }
        PP_HIP(hipStreamSynchronize(H->stream));
        return PP_OK;
    });
}

int pp_destroy(pp_handle h)
{
    if (!h) return PP_OK;
    Handle* H = &h->h;
    (void)hipSetDevice(H->device);
    if (H->stream) (void)hipStreamSynchronize(H->stream);
    if (H->side) (void)hipStreamSynchronize(H->side);
    if (H->arena) (void)hipFree(H->arena);
    if (H->host_slots) (void)hipHostFree(H->host_slots);
    if (H->ev0) (void)hipEventDestroy(H->ev0);
    if (H->ev1) (void)hipEventDestroy(H->ev1);
    for (hipEvent_t e : H->ev_pool) (void)hipEventDestroy(e);
    drop_graphs(H);
    if (H->stream) (void)hipStreamDestroy(H->stream);
    if (H->side) (void)hipStreamDestroy(H->side);
    if (H->ev_coarse) (void)hipEventDestroy(H->ev_coarse);
    if (H->ev_dense) (void)hipEventDestroy(H->ev_dense);
    if (H->ev_in) (void)hipEventDestroy(H->ev_in);
    if (H->ev_out) (void)hipEventDestroy(H->ev_out);
    delete h;
    return PP_OK;
}

int pp_kernel_timing(pp_handle h, int mode, pp_kernel_time* out, int max_entries)
{
    if (!h) { g_thread_err = "null handle"; return PP_ERR_INVALID; }
    Handle* H = &h->h;
    if (mode == 1 || mode == -1) {
        // graphs are recaptured with (or without) event nodes on their next use
        (void)hipStreamSynchronize(H->stream);
        drop_graphs(H);
        if (mode == 1)
            for (int i = 0; i < 64; ++i) { H->kt_ms[i] = 0.0; H->kt_bytes[i] = 0.0; H->kt_count[i] = 0; }
        H->timing = mode == 1;
        return 0;
    }
    int n = 0;
    for (int prec = 0; prec < 2; ++prec)
        for (int k = 0; k < KT_N; ++k) {
            int id = k + 32 * prec;
            if (H->kt_count[id] == 0) continue;
            if (out && n < max_entries) {
                std::snprintf(out[n].name, sizeof(out[n].name), "%s_%s", kt_name[k], prec ? "f64" : "f32");
                out[n].total_ms = H->kt_ms[id];
                out[n].launches = H->kt_count[id];
                out[n].bytes = H->kt_bytes[id];
            }
            ++n;
        }
    return out ? std::min(n, max_entries) : n;
}

const char* pp_last_error(pp_handle h)
{
    if (h) return h->h.err.c_str();
    return g_thread_err.c_str();
}

int pp_density_from_fraction(const double* a, double rho_l, double rho_g, double* rho, size_t n, void* hip_stream)
{
    if (!a || !rho) { g_thread_err = "null pointer"; return PP_ERR_INVALID; }
    return guarded(nullptr, [&]() -> int {
        if (n == 0) return PP_OK;
        k_density<<<lin_grid(n), kBlock, 0, (hipStream_t)hip_stream>>>(n, a, rho_l, rho_g, rho);
        check_launch();
        PP_HIP(hipStreamSynchronize((hipStream_t)hip_stream));
        return PP_OK;
    });
}

int pp_divergence(int nx, int ny, int nz, double h, double dt, const double* u, const double* v, const double* w, double* out,
                  void* hip_stream)
{
    if (!u || !v || !w || !out) { g_thread_err = "null pointer"; return PP_ERR_INVALID; }
    if (nx < 1 || ny < 1 || nz < 1 || !(h > 0.0) || !(dt > 0.0) || !grid_fits_int(nx, ny, nz)) {
        g_thread_err = "bad sizes, h or dt";
        return PP_ERR_INVALID;
    }
    return guarded(nullptr, [&]() -> int {
        Geo g = geo(nx, ny, nz, 8192);
        k_divergence<<<g.grid, g.block, 0, (hipStream_t)hip_stream>>>(nx, ny, nz, h * dt, u, v, w, out, g.kper);
        check_launch();
        PP_HIP(hipStreamSynchronize((hipStream_t)hip_stream));
        return PP_OK;
    });
}

int pp_project(int nx, int ny, int nz, double h, double dt, const double* rho, const double* p, double* u, double* v, double* w,
               void* hip_stream)
{
    if (!rho || !p || !u || !v || !w) { g_thread_err = "null pointer"; return PP_ERR_INVALID; }
    if (nx < 1 || ny < 1 || nz < 1 || !(h > 0.0) || !(dt > 0.0) || !grid_fits_int(nx, ny, nz)) {
        g_thread_err = "bad sizes, h or dt";
        return PP_ERR_INVALID;
    }
    return guarded(nullptr, [&]() -> int {
        Geo g = geo(nx, ny, nz, 8192);
        k_project<<<g.grid, g.block, 0, (hipStream_t)hip_stream>>>(nx, ny, nz, h, dt, rho, p, u, v, w, g.kper);
        check_launch();
        PP_HIP(hipStreamSynchronize((hipStream_t)hip_stream));
        return PP_OK;
    });
}

int pp_rel_residual(int nx, int ny, int nz, double h, const double* rho, const double* rhs, const double* p, double* rel_out,
                    void* hip_stream)
{
    if (int e = rel_residual_args(nx, ny, nz, h, rho, rhs, p, rel_out)) return e;
    double* buf = nullptr;
    const size_t bytes = sizeof(double) * ((size_t)kMaxPartialBlocks * kMaxRed + kRelSlots);
    int rc = guarded(nullptr, [&]() -> int {
        hipError_t e = hipMalloc((void**)&buf, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            buf = nullptr;
            throw Fail(PP_ERR_OOM, "hipMalloc of the residual's partial sums failed");
        }
        return rel_residual_on((hipStream_t)hip_stream, nx, ny, nz, h, rho, rhs, p, rel_out, buf,
                               buf + (size_t)kMaxPartialBlocks * kMaxRed);
    });
    if (buf) {
        (void)hipStreamSynchronize((hipStream_t)hip_stream);
        (void)hipFree(buf);
    }
    return rc;
}

int pp_rel_residual_noalloc(int nx, int ny, int nz, double h, const double* rho, const double* rhs, const double* p,
                            double* rel_out, void* hip_stream)
{
    if (int e = rel_residual_args(nx, ny, nz, h, rho, rhs, p, rel_out)) return e;
    return guarded(nullptr, [&]() -> int {
        double* buf = scratch_of_current_device();
        return rel_residual_on((hipStream_t)hip_stream, nx, ny, nz, h, rho, rhs, p, rel_out, buf,
                               buf + (size_t)kMaxPartialBlocks * kMaxRed);
    });
}

int pp_correct_velocity(int nx, int ny, int nz, double h, double dt, const double* rho, const double* p, const double* pt,
                        double* u, double* v, double* w, double* uc, double* vc, double* wc, void* hip_stream)
{
    if (!rho || !p || !u || !v || !w || !uc || !vc || !wc) { g_thread_err = "null pointer"; return PP_ERR_INVALID; }
    if (nx < 1 || ny < 1 || nz < 1 || !(h > 0.0) || !(dt > 0.0) || !grid_fits_int(nx, ny, nz)) {
        g_thread_err = "bad sizes, h or dt";
        return PP_ERR_INVALID;
    }
    return guarded(nullptr, [&]() -> int {
        Geo g = geo(nx, ny, nz, 8192);
        if (pt)
            k_correct_velocity<true><<<g.grid, g.block, 0, (hipStream_t)hip_stream>>>(nx, ny, nz, h, dt, rho, p, pt, u, v, w,
                                                                                      uc, vc, wc, g.kper);
        else
            k_correct_velocity<false><<<g.grid, g.block, 0, (hipStream_t)hip_stream>>>(nx, ny, nz, h, dt, rho, p, pt, u, v,
                                                                                       w, uc, vc, wc, g.kper);
        check_launch();
        PP_HIP(hipStreamSynchronize((hipStream_t)hip_stream));
        return PP_OK;
    });
}

int pp_surface_tension_rhs(int nx, int ny, int nz, double h, double sigma, const double* rho, const double* alpha,
                           const double* kappa, double* out, void* hip_stream)
{
    if (!rho || !alpha || !kappa || !out) { g_thread_err = "null pointer"; return PP_ERR_INVALID; }
    if (nx < 1 || ny < 1 || nz < 1 || !(h > 0.0) || !grid_fits_int(nx, ny, nz)) {
        g_thread_err = "bad sizes or h";
        return PP_ERR_INVALID;
    }
    return guarded(nullptr, [&]() -> int {
        Geo g = geo(nx, ny, nz, 8192);
        k_surface_rhs<<<g.grid, g.block, 0, (hipStream_t)hip_stream>>>(nx, ny, nz, h, sigma, rho, alpha, kappa, out, g.kper);
        check_launch();
        PP_HIP(hipStreamSynchronize((hipStream_t)hip_stream));
        return PP_OK;
    });
}

}  // extern "C"
