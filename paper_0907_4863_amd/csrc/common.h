// Internal declarations of the SA-AMG PCG library (not part of the C interface).
//
// Data layout on the device
//   Level 0 (the lattice): box vectors of nx*ny*nz values, x fastest.  The scaled
//   operator D^-1/2 A D^-1/2 has unit diagonal.  Rows of interior points whose six
//   off-diagonals all equal the interior constants (-sigma0^2/h_a^2) are "regular"; the
//   others ("irregular": rows with an outside neighbour, and the neighbours of rows
//   with a cut wall) keep their six coefficients in a compact table.  Per 64-node
//   segment of an x-line the library stores a 64-bit unknown mask, a 64-bit irregular
//   mask and the table rank of the segment's first irregular row, so a row's table
//   slot is base + popcount(irregular bits below it).
//   Levels >= 1: 27-point Galerkin operators on a logical box (mx, my, mz) stored with a
//   one-node zero ghost layer, i.e. on (mx+2)*(my+2)*(mz+2) nodes; coefficient k of
//   row i couples i to i + offset(k), k = (dx+1) + 3(dy+1) + 9(dz+1).  A symmetric
//   operator stores only k >= 13 and reads A(i, k<13) as A(i+off(k), 26-k).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/saamg.h"
#include "host_prep.h"

namespace saamg {

constexpr int kWave = 64;
constexpr int kBlockY = 4;          // 64 x 4 threads per block for box kernels
constexpr int kThreads = kWave * kBlockY;
constexpr long kGsMax = 8192;     // coarsest-level storage for the Gauss-Seidel solver (LDS)
constexpr int kMY = 4;              // wavefronts per block of the level-0 solve-time kernels
constexpr int kMThreads = kWave * kMY;
constexpr int kFinThreads = 1024;   // single-block finalisation of partial sums

// Direction d = 0..5 (-x,+x,-y,+y,-z,+z) as a 27-point offset index.
__host__ __device__ constexpr int dir_to_k(int d) {
    return d == 0 ? 12 : d == 1 ? 14 : d == 2 ? 10 : d == 3 ? 16 : d == 4 ? 4 : 22;
}

template <typename T>
struct L0View {
    int nx, ny, nz, nsegx;
    int tx, gx, gy, zb; // solve-time tiling: segments per block along x, block columns,
                        // block rows (kMY / tx lines each), planes per block
    long nxy;
    const uint64_t* unk;
    const uint64_t* irr;
    const int32_t* base;
    // scaled off-diagonals of the irregular rows: table slot r holds 8 values, the 6
    // directions and 2 of padding, so that a row is read with two 16-byte loads (fp32) or
    // three (fp64) instead of one load per direction; tabT holds the same rows of the
    // transpose
    const T* tab;
    const T* tabT;
    __host__ __device__ T tcoef(int d, long r) const { return tab[8 * r + d]; }
    __host__ __device__ T tcoefT(int d, long r) const { return tabT[8 * r + d]; }
    T c[3];             // interior off-diagonal per axis
    double rho_end;     // factor of the end-plane rows (1/2 with open ends, else 1)
    const double* skip; // nonzero *skip: the kernel returns at once (see g_vskip)
};

// Values per row of a level >= 1 coefficient table (27 and 1 of padding).
constexpr int kLcRow = 28;

// A level >= 1 operator.  The solve kernels read it compressed: a node's row is the
// level's interior stencil (slot -1), zero (slot -2: not an unknown or a ghost), or row
// `slot` of the table.  The full per-offset arrays (fp64 views only) serve setup and
// diagnostics.
template <typename T>
struct LCView {
    int mx, my, mz;     // logical box
    int sx, sy;         // storage pitch (mx+2, my+2)
    long sxy;
    long off[27];
    const T* coef[27];  // full fp64 arrays, storage layout; symmetric: coef[k<13] = nullptr
    const T* invD;      // 1/diag, 0 at nodes that are not unknowns and in the ghost layer
    int sym;
    const int32_t* slot;  // per storage node
    T cst[27];            // the interior stencil
    // nonsymmetric levels: the transpose, compressed the same way (slot -1: the node and
    // its 26 neighbours all have the interior row, so A^T(i, k) = cst[26 - k])
    const int32_t* slotT;
    // table rows: tb[kLcRow * s + k] = A(i, i + off[k]) for the node of slot s (tbT: the
    // transpose); kLcRow = 28 values per row (27 and 1 of padding), so that a row is read
    // with 16-byte loads
    const T* tb;
    const T* tbT;
    long tcap, tTcap;     // rows allocated
    const double* skip;   // nonzero *skip: the kernel returns at once (see g_vskip)
};

// ---------------------------------------------------------------- device helpers

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, kWave);
    return v;
}

// Sum over a block of blockDim.x*blockDim.y threads (multiple of 64); result in thread 0.
__device__ inline double block_sum(double v, double* lds) {
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    const int nw = (blockDim.x * blockDim.y) / kWave;
    v = wave_sum(v);
    if ((tid & (kWave - 1)) == 0) lds[tid / kWave] = v;
    __syncthreads();
    double s = 0.0;
    if (tid == 0) {
        for (int w = 0; w < nw; ++w) s += lds[w];
    }
    __syncthreads();
    return s;
}

__device__ inline long block_linear_id() {
    return blockIdx.x + (long)gridDim.x * (blockIdx.y + (long)gridDim.y * blockIdx.z);
}

__device__ inline long grid_blocks() { return (long)gridDim.x * gridDim.y * gridDim.z; }

// Lanczos start value of a logical box index: output number lin of SplitMix64 from
// state 0 (Steele, Lea, Flood, OOPSLA 2014), its top 53 bits mapped to [-1/2, 1/2).
__host__ __device__ inline double start_value(long lin) {
    uint64_t z = ((uint64_t)lin + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1.0p-53 - 0.5;
}

// ---------------------------------------------------------------- host side

struct HipError {
    hipError_t e;
    std::string where;
};

void hip_check(hipError_t e, const char* what);

// Device allocator of a hierarchy (the options' callbacks; both null: hipMalloc / hipFree)
// and the stream on which an entry point queues its work.
struct MemCtx {
    void* (*alloc)(void*, size_t, void*) = nullptr;
    void (*free)(void*, void*, void*) = nullptr;
    void* ctx = nullptr;
    hipStream_t s = nullptr;
    bool fill = true;  // zero-fill new buffers (off only for a pass that measures sizes)
};
// Makes (m, s) the allocator and fill stream of dmalloc / dfree on the calling thread for
// the scope's lifetime.
struct MemScope {
    MemCtx saved;
    MemScope(const MemCtx& m, hipStream_t s);
    ~MemScope();
    MemScope(const MemScope&) = delete;
    MemScope& operator=(const MemScope&) = delete;
};
#define HIPCHECK(x) ::saamg::hip_check((x), #x)

// While a solve's preconditioner is queued, the device address of its skip flag: every
// view built then carries it, and the V-cycle's kernels return at once when the flag is
// nonzero.  The flag is set on the device by the test of the residual the V-cycle would
// precondition, when that residual already passes the stopping rule (the host would
// discard the result).  Null elsewhere (setup, diagnostics, the CG kernels).
extern thread_local const double* g_vskip;
struct VSkipScope {
    const double* saved;
    explicit VSkipScope(const double* flag) : saved(g_vskip) { g_vskip = flag; }
    ~VSkipScope() { g_vskip = saved; }
    VSkipScope(const VSkipScope&) = delete;
    VSkipScope& operator=(const VSkipScope&) = delete;
};

// Allocates through the thread's MemScope and zero-fills on its stream (stream-ordered);
// throws ApiError(NOMEM) on failure.
void* dmalloc(size_t bytes);
void dfree(void* p);

// A temporary device buffer of one step, returned to the allocator when the step's scope
// ends, also when an exception leaves it.  The step synchronises its stream before a
// normal exit; an allocator's stream-ordered reuse covers the exceptional one.
struct Tmp {
    void* p = nullptr;
    explicit Tmp(size_t bytes) : p(dmalloc(bytes)) {}
    ~Tmp() { dfree(p); }
    Tmp(const Tmp&) = delete;
    Tmp& operator=(const Tmp&) = delete;
    template <typename T>
    T* as() const { return (T*)p; }
};

// Opt-in kernel timing of one kernel class (see saamg_timer_* in the C interface).  A
// timer spans one launch function: its first launch carries the start event and its last
// the stop event, so the timestamps are those of the kernel dispatches themselves and no
// marker is added to the stream between kernels.
enum TimerKind {
    T_L0_CHEB = 0, T_L0_RESID, T_L0_RESTRICT, T_L0_PROLONG, T_CG_PQ, T_CG_XR, T_COARSE,
    T_FINALIZE, T_CG_X, T_NKIND
};
struct KTimer {
    int slot = -1;
    int kind;
    hipStream_t s;
    bool started = false, stopped = false;
    KTimer(int kind, hipStream_t s, long units);
    hipEvent_t start();  // the start event for the first launch (null when off or taken)
    hipEvent_t stop();   // the stop event (null when off)
    ~KTimer();           // records the events that no launch carried
};

// Launches kernel f on the timer's stream; `last` marks the timer's final launch.
template <typename F, typename... Args>
inline void klaunch(KTimer& kt, bool last, F f, dim3 grid, dim3 block, Args... args) {
    hipExtLaunchKernelGGL(f, grid, block, 0, kt.s, kt.start(), last ? kt.stop() : nullptr, 0,
                          args...);
}

struct ChebCoef {
    int degree;
    double c1[8];   // multiplies the previous direction
    double c2[8];   // multiplies D^-1 r
};
ChebCoef cheb_coefficients(double lam_hi, double ratio, int degree);

struct FineLevel {
    int nx, ny, nz, nsegx;
    int zb = 4;                 // planes per block of the solve-time kernels
    int tx = 1;                 // segments per block along x of the solve-time kernels
    // 16-byte lanes (wide.hip): the V-cycle and CG kernels run with 4 (fp32) or 2 (fp64)
    // nodes per lane; wzb[0] / wzb[1]: their planes per block with 2 / 4 nodes per lane
    int wide = 0;
    int wzb[2] = {2, 2};
    long nxy, nbox, nseg;
    double h[3];
    uint64_t* unk = nullptr;
    uint64_t* irr = nullptr;
    int32_t* base = nullptr;    // table slot of each segment's first irregular row
    int32_t* base_full = nullptr;  // the same before de-duplication (one row per node)
    long n_irr = 0;             // irregular rows
    long n_tab = 0;             // table rows: lines repeating the line one plane below share
                                // its rows (see l0_dedup_table)
    double* tab64 = nullptr;    // [2][n_tab][8]: rows of the operator, then of its transpose
    float* tab32 = nullptr;
    double c64[3];
    double robin_d = 0.0;       // open ends (Robin parameter d); 0: closed ends
    double* sigma = nullptr;    // box, D^-1/2 at unknowns
    long n_unknowns = 0;

    template <typename T>
    L0View<T> view() const;
};

struct CoarseLevel {
    int mx, my, mz;
    int sx, sy, sz;
    long sxy, nstore;
    int sym;
    double* coef64[27] = {};
    double* invD64 = nullptr;
    double* block64 = nullptr;  // one allocation holding the coef64 arrays and invD64
    float* invD32 = nullptr;
    long n_unknowns = 0;
    // compressed operator: slot per storage node, interior stencil, table [tab_cap][kLcRow]
    int32_t* slot = nullptr;
    double cst64[27] = {};
    long n_tab = 0, tab_cap = 0;
    double* tab64 = nullptr;
    float* tab32 = nullptr;
    // transpose (nonsymmetric levels only)
    int32_t* slotT = nullptr;
    long n_tabT = 0, tabT_cap = 0;
    double* tabT64 = nullptr;
    float* tabT32 = nullptr;

    template <typename T>
    LCView<T> view() const;
};

struct LevelParams {
    double lam = 0, lam_hi = 0, omega = 0;
    ChebCoef cheb{};
};

}  // namespace saamg

struct saamg_hierarchy {
    int device = 0;
    saamg::MemCtx mem;        // allocator of every buffer of the hierarchy and its states
    int variant = 1;
    saamg_options opt{};
    int sym = 1;
    int n_levels = 1;
    saamg::FineLevel l0{};
    // the CG iteration's level-0 operator when it differs from the preconditioner's
    // (saamg_set_operator): own table and scaling, the segment masks of l0; else null
    saamg::FineLevel* op = nullptr;
    std::vector<saamg::CoarseLevel> lc;     // lc[l-1] is level l
    std::vector<saamg::LevelParams> par;    // per level except the coarsest
    // coarsest level: explicit inverse, fp64, and where its unknowns live
    int nL = 0;
    double* Ainv = nullptr;
    long* cidx = nullptr;     // storage index of each coarsest-level unknown
    double t_setup_ms = 0;
    double t_phase_ms[6] = {};  // setup phases (see saamg_info.t_setup_phase_ms)
    double t_refresh_ms = 0;  // last saamg_refresh, 0 if none
    int live_states = 0;      // saamg_state objects created on H and not yet destroyed
    int64_t bytes = 0;
    // work vectors of saamg_solve / saamg_precond_apply, allocated on first use
    saamg_state* ws = nullptr;
};

namespace saamg {
// Segments of one line that a block of the level-0 solve-time kernels covers (its other
// wavefronts take the next lines): whole 256-node lines where the box is wide enough
// (the automatic choice; an option may ask for fewer).
inline int l0_tile_x(int nsegx) { return nsegx >= kMY ? kMY : (nsegx >= 2 ? 2 : 1); }

template <typename T>
inline L0View<T> FineLevel::view() const {
    L0View<T> v;
    v.nx = nx; v.ny = ny; v.nz = nz; v.nsegx = nsegx; v.nxy = nxy;
    v.tx = tx;
    v.gx = (nsegx + v.tx - 1) / v.tx;
    v.gy = (ny + kMY / v.tx - 1) / (kMY / v.tx);
    v.zb = zb;
    v.unk = unk; v.irr = irr; v.base = base;
    if constexpr (sizeof(T) == 8) {
        v.tab = (const T*)tab64;
        v.tabT = (const T*)(tab64 ? tab64 + 8 * n_tab : nullptr);
    } else {
        v.tab = (const T*)tab32;
        v.tabT = (const T*)(tab32 ? tab32 + 8 * n_tab : nullptr);
    }
    for (int a = 0; a < 3; ++a) v.c[a] = (T)c64[a];
    v.rho_end = robin_d > 0.0 ? 0.5 : 1.0;
    v.skip = g_vskip;
    return v;
}

template <typename T>
inline LCView<T> CoarseLevel::view() const {
    LCView<T> v;
    v.mx = mx; v.my = my; v.mz = mz; v.sx = sx; v.sy = sy; v.sxy = sxy; v.sym = sym;
    v.slot = slot;
    v.slotT = slotT;
    for (int k = 0; k < 27; ++k) {
        int dx = k % 3 - 1, dy = (k / 3) % 3 - 1, dz = k / 9 - 1;
        v.off[k] = dx + (long)sx * dy + sxy * dz;
        v.cst[k] = (T)cst64[k];
        v.coef[k] = sizeof(T) == 8 ? (const T*)coef64[k] : nullptr;
    }
    if constexpr (sizeof(T) == 8) {
        v.invD = invD64;
        v.tb = tab64;
        v.tbT = tabT64;
    } else {
        v.invD = invD32;
        v.tb = tab32;
        v.tbT = tabT32;
    }
    v.tcap = tab_cap;
    v.tTcap = tabT_cap;
    v.skip = g_vskip;
    return v;
}
}  // namespace saamg
