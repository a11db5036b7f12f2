// Kernels of levels >= 1 (27-point Galerkin operators on ghost-padded boxes), the
// structured Galerkin product that builds them, the compression the solve kernels read
// them in (interior stencil, per-node slot, table of the other rows; also for the
// transpose of nonsymmetric levels), and the coarsest-level solvers.
#include "march.h"

namespace saamg {

// Coefficient k of the row with slot s (compressed operator).
template <typename T>
__device__ inline T lc_row(const LCView<T>& c, int s, int k) {
    return s >= 0 ? c.tb[(long)kLcRow * s + k] : (s == -1 ? c.cst[k] : T(0));
}
// Coefficient A(i, k) of a 27-point level.
template <typename T, bool SYM>
__device__ inline T lc_a(const LCView<T>& c, long i, int k) {
    return lc_row(c, c.slot[i], k);
}
// Coefficient k of the transpose row with slot s: A^T(i, k) = A(i + off(k), 26 - k).
template <typename T>
__device__ inline T lc_rowT(const LCView<T>& c, int s, int k) {
    return s >= 0 ? c.tbT[(long)kLcRow * s + k] : (s == -1 ? c.cst[26 - k] : T(0));
}
template <typename T, bool SYM>
__device__ inline T lc_at(const LCView<T>& c, long i, int k) {
    if (SYM) return lc_a<T, true>(c, i, k);
    return lc_rowT(c, c.slotT[i], k);
}

// Row s of a coefficient table into t: 7 (fp32) or 14 (fp64) 16-byte loads.
template <typename T>
__device__ __forceinline__ void lc_load_row(const T* tb, int s, T (&t)[kLcRow]) {
    if constexpr (sizeof(T) == 4) {
        const float4* p = reinterpret_cast<const float4*>(tb + (long)kLcRow * s);
#pragma unroll
        for (int q = 0; q < kLcRow / 4; ++q) {
            const float4 v = p[q];
            t[4 * q] = v.x;
            t[4 * q + 1] = v.y;
            t[4 * q + 2] = v.z;
            t[4 * q + 3] = v.w;
        }
    } else {
        const double2* p = reinterpret_cast<const double2*>(tb + (long)kLcRow * s);
#pragma unroll
        for (int q = 0; q < kLcRow / 2; ++q) {
            const double2 v = p[q];
            t[2 * q] = v.x;
            t[2 * q + 1] = v.y;
        }
    }
}

// Storage offset of neighbour k, from the pitches (the unrolled loops fold the constants).
template <typename T>
__device__ inline long lc_off(const LCView<T>& c, int k) {
    return (k % 3 - 1) + (long)c.sx * ((k / 3) % 3 - 1) + c.sxy * (k / 9 - 1);
}

// sum_k A(i, k) X(i + off_k) (TR: A^T), offsets in order k = 0..26.  A wavefront whose
// lanes are all interior rows takes the stencil from registers; one that holds any table
// row runs a single loop that picks each lane's coefficient, so the neighbour values are
// loaded once per offset whatever the mix of rows in the wavefront.
template <typename T, bool SYM, bool TR, class F>
__device__ inline T lc_stencil(const LCView<T>& c, long i, F X) {
    constexpr bool kT = TR && !SYM;
    const int s = kT ? c.slotT[i] : c.slot[i];
    if (s == -2) return T(0);
    T acc = 0;
    if (__ballot(s >= 0) == 0) {
#pragma unroll
        for (int k = 0; k < 27; ++k) acc += c.cst[kT ? 26 - k : k] * X(i + lc_off(c, k));
        return acc;
    }
    const int sc = s < 0 ? 0 : s;  // a valid table row for the interior lanes' (unused) load
    T t[kLcRow];
    lc_load_row(kT ? c.tbT : c.tb, sc, t);
#pragma unroll
    for (int k = 0; k < 27; ++k) acc += (s >= 0 ? t[k] : c.cst[kT ? 26 - k : k]) * X(i + lc_off(c, k));
    return acc;
}

// A(i, k) from the full fp64 arrays (setup).
__device__ inline double lc_full(const LCView<double>& c, long i, int k) {
    return (c.sym && k < 13) ? c.coef[26 - k][i + c.off[k]] : c.coef[k][i];
}

static inline dim3 lc_grid(const CoarseLevel& C) {
    return dim3((unsigned)(((long)C.mx * C.my + kThreads - 1) / kThreads), C.mz);
}
long lc_blocks(const CoarseLevel& C) {
    dim3 g = lc_grid(C);
    return (long)g.x * g.y * g.z;
}

// One thread per node of a z-plane (flattened over x and y so that wavefronts stay full
// on narrow coarse boxes), one block row per plane.
#define LC_PROLOGUE                                                              \
    if (c.skip && *c.skip != 0.0) return;                                        \
    const long t_ = blockIdx.x * (long)blockDim.x + threadIdx.x;                 \
    const bool inb = t_ < (long)c.mx * c.my;                                     \
    const int X = inb ? (int)(t_ % c.mx) : 0;                                    \
    const int Y = inb ? (int)(t_ / c.mx) : 0;                                    \
    const int Z = blockIdx.y;                                                    \
    const long i = (X + 1) + (long)c.sx * (Y + 1) + c.sxy * (Z + 1);

// ---------------------------------------------------------------- solve-time z-march
//
// The solve kernels of levels >= 1 march along z like the level-0 ones.  A wavefront owns
// kLcSeg = 62 consecutive nodes of one line (storage x = 62 s + lane in segment s; lanes 0
// and 63 are its halo, which only load), keeps X at the 3 x 3 (y, z) neighbour columns of
// its node in registers, takes the x-neighbours from the adjacent lanes and loads 3 values
// per plane (the next plane's rows y-1, y, y+1) where one thread per node loads 27.  The
// plane's loads (its slot, the kernel's operands, the next plane's rows) are issued a
// plane ahead; a row that is not the interior stencil reads its table row in the step.
// The stencil sums its 27 terms in the order k = 0..26, as lc_stencil does.
constexpr int kLcSeg = kWave - 2;

struct LcTile {
    int tx, gx, gy, zb;  // segments per block along x, block columns, block rows, planes
};

static LcTile lc_tiling(const CoarseLevel& C) {
    LcTile t;
    const int nsx = (C.mx + kLcSeg - 1) / kLcSeg;
    t.tx = nsx >= kMY ? kMY : (nsx >= 2 ? 2 : 1);
    t.gx = (nsx + t.tx - 1) / t.tx;
    t.gy = (C.my + kMY / t.tx - 1) / (kMY / t.tx);
    // long z-runs where the level is large, down to 2 planes on the small levels
    const long tiles = (long)t.gx * t.gy;
    t.zb = 8;
    while (t.zb > 2 && tiles * ((C.mz + t.zb - 1) / t.zb) < 2048) t.zb /= 2;
    return t;
}
static inline dim3 lc_mgrid(const CoarseLevel& C, const LcTile& t) {
    return dim3((unsigned)((long)t.gx * t.gy * ((C.mz + t.zb - 1) / t.zb)));
}

// Segment, line and z-slab of this wavefront (the XCD-aware remap of l0_tile).
__device__ inline void lc_tile(const LcTile& t, int* seg, int* Y, int* bz) {
    const unsigned b = blockIdx.x, nb = gridDim.x;
    const unsigned q = nb >> 3;
    const unsigned lb = (b < 8 * q) ? (b & 7) * q + (b >> 3) : b;
    const int w = threadIdx.y;
    const unsigned tt = lb / (unsigned)t.gx;
    *seg = (int)(lb % (unsigned)t.gx) * t.tx + w % t.tx;
    *Y = (int)(tt % (unsigned)t.gy) * (kMY / t.tx) + w / t.tx;
    *bz = (int)(tt / (unsigned)t.gy);
}

template <typename T, class FV>
struct LcPlane {
    T nxt[3];  // X at the next plane, rows y-1, y, y+1
    int slot;  // this plane's slot (of A, or of A^T when transposed)
    FV fv;
};

// March of a tile.  For every node of the tile the march calls
//   fv = fetch(i)                         (loads, issued a plane ahead)
//   body(i, fv, xc, ax, comp)             (arithmetic and stores)
// with the storage index i, X at the node (xc) and ax = (A X)_i (TR: A^T X; 0 where the
// slot is -2); comp is false on the halo lanes and past the box, whose i must not be
// written.  X(i, xs, ys, zs) returns X at storage index i = xs + sx ys + sxy zs (the
// coordinates for loaders that gather, such as the prolongation's coarse values).
template <typename T, bool SYM, bool TR, class Load, class Fetch, class Body>
__device__ __forceinline__ void lc_march(const LCView<T>& c, const LcTile& tl, Load X, Fetch fetch,
                                         Body body) {
    constexpr bool kT = TR && !SYM;
    using FV = decltype(fetch(0L));
    using P = LcPlane<T, FV>;
    if (c.skip && *c.skip != 0.0) return;  // wave-uniform: the whole grid returns
    int seg, Y, bz;
    lc_tile(tl, &seg, &Y, &bz);
    seg = __builtin_amdgcn_readfirstlane(seg);
    Y = __builtin_amdgcn_readfirstlane(Y);
    const int lane = threadIdx.x;
    const int nsx = (c.mx + kLcSeg - 1) / kLcSeg;
    if (Y >= c.my || seg >= nsx) return;
    const int Z0 = bz * tl.zb, Z1 = min(Z0 + tl.zb, c.mz);
    if (Z0 >= Z1) return;
    const int xs = min(seg * kLcSeg + lane, c.mx + 1);  // storage x, clamped to the ghost
    const bool comp = lane >= 1 && lane <= kLcSeg && seg * kLcSeg + lane <= c.mx;
    const int ys = Y + 1;
    const long sx = c.sx, sxy = c.sxy;
    const long rb = xs + sx * ys;  // storage index of the lane's column at storage plane 0
    const int32_t* slots = kT ? c.slotT : c.slot;
    const T* tbl = kT ? c.tbT : c.tb;
    auto load_plane = [&](int zs) {  // storage plane zs (the node plane)
        P p;
        const long i = rb + sxy * zs, n = i + sxy;
        p.nxt[0] = X(n - sx, xs, ys - 1, zs + 1);
        p.nxt[1] = X(n, xs, ys, zs + 1);
        p.nxt[2] = X(n + sx, xs, ys + 1, zs + 1);
        p.slot = slots[i];
        p.fv = fetch(i);
        return p;
    };
    T col[3][3];  // [dz][dy] at the lane's x: planes zs-1, zs, zs+1
    {
        const long i0 = rb + sxy * Z0;  // storage plane Z0 = the plane below the first node
#pragma unroll
        for (int dz = 0; dz < 2; ++dz)
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
                col[dz][dy] = X(i0 + sxy * dz + sx * (dy - 1), xs, ys + dy - 1, Z0 + dz);
    }
    // The lane's table row stays in registers from plane to plane and is read again only
    // when its slot changes: table rows equal to the row one plane below share its slot, so
    // along a pipe of constant cross-section most planes read no table row at all.
    T t[kLcRow];
#pragma unroll
    for (int k = 0; k < kLcRow; ++k) t[k] = T(0);
    int held = -1;  // slot whose row t holds
    auto step = [&](const P& p, int Z) {
        settle(p.nxt);
        settle(p.slot);
        settle(p.fv);
        if (Z >= Z1) return;
        const long i = rb + sxy * (Z + 1);
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) col[2][dy] = p.nxt[dy];
        const int s = p.slot;
        const bool need = s >= 0 && s != held;
        if (__ballot(need) != 0) {
            if (need) {
                lc_load_row(tbl, s, t);
                held = s;
            }
        }
        T acc = T(0);
#pragma unroll
        for (int k = 0; k < 27; ++k) {
            const int dx = k % 3 - 1, dy = (k / 3) % 3, dz = k / 9;
            const T v0 = col[dz][dy];
            const T xv = dx == 0 ? v0 : (dx < 0 ? wave_shift<true>(v0, T(0)) : wave_shift<false>(v0, T(0)));
            const T a = s >= 0 ? t[k] : c.cst[kT ? 26 - k : k];
            acc += a * xv;
        }
        if (s == -2) acc = T(0);
        body(i, p.fv, col[1][1], acc, comp);
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
            col[0][dy] = col[1][dy];
            col[1][dy] = col[2][dy];
        }
    };
    P pa = load_plane(Z0 + 1);
    for (int Z = Z0; Z < Z1; Z += 2) {
        P pb = load_plane(min(Z + 2, Z1));
        step(pa, Z);
        pa = load_plane(min(Z + 3, Z1));
        step(pb, Z + 1);
    }
}

// Loader of X from a storage vector.
#define LC_LOAD(p) [&](long j, int, int, int) { return (p)[j]; }

template <typename T, bool SYM, bool TR>
__global__ void __launch_bounds__(kMThreads) k_lc_apply(LCView<T> c, LcTile tl,
                                                        const T* __restrict__ xv,
                                                        T* __restrict__ yv) {
    lc_march<T, SYM, TR>(c, tl, LC_LOAD(xv), [&](long) { return 0; },
                         [&](long i, int, T, T ax, bool comp) {
                             if (comp) yv[i] = ax;
                         });
}

template <typename T>
void lc_apply(const CoarseLevel& C, bool trans, const T* x, T* y, hipStream_t s) {
    LCView<T> c = C.view<T>();
    const LcTile tl = lc_tiling(C);
    const dim3 g = lc_mgrid(C, tl), b(kWave, kMY);
    if (C.sym)
        hipLaunchKernelGGL((k_lc_apply<T, true, false>), g, b, 0, s, c, tl, x, y);
    else if (trans)
        hipLaunchKernelGGL((k_lc_apply<T, false, true>), g, b, 0, s, c, tl, x, y);
    else
        hipLaunchKernelGGL((k_lc_apply<T, false, false>), g, b, 0, s, c, tl, x, y);
    HIPCHECK(hipGetLastError());
}
template void lc_apply<double>(const CoarseLevel&, bool, const double*, double*, hipStream_t);
template void lc_apply<float>(const CoarseLevel&, bool, const float*, float*, hipStream_t);

// Lanczos in the D inner product (see the level-0 version for the storage of vectors).

// v = start vector at the unknowns; partials of v.(D v).
__global__ void __launch_bounds__(kThreads) k_lc_lz_start(LCView<double> c, double* w,
                                                         double* part) {
    __shared__ double lds[kThreads / kWave];
    LC_PROLOGUE
    double a0 = 0.0;
    if (inb) {
        const long lin = X + (long)c.mx * (Y + (long)c.my * Z);
        const double id = c.invD[i];
        const double sv = id != 0.0 ? start_value(lin) : 0.0;
        w[i] = sv;
        if (id != 0.0) a0 = sv * sv / id;
    }
    const double s0 = block_sum(a0, lds);
    if (threadIdx.x == 0 && threadIdx.y == 0) part[block_linear_id()] = s0;
}

void lc_lz_start(const CoarseLevel& C, double* v, double* partials, hipStream_t s) {
    hipLaunchKernelGGL(k_lc_lz_start, lc_grid(C), dim3(kThreads), 0, s, C.view<double>(), v,
                       partials);
    HIPCHECK(hipGetLastError());
}

// u = S q, q = vin * scal[S_LZ_S], S = (A + A^T)/2; partials of q.u.
template <bool SYM>
__global__ void __launch_bounds__(kThreads) k_lc_lz_apply(LCView<double> c,
                                                         const double* __restrict__ vin,
                                                         const double* __restrict__ scal,
                                                         double* __restrict__ u, double* part) {
    __shared__ double lds[kThreads / kWave];
    const double sc = scal[S_LZ_S];
    LC_PROLOGUE
    double a0 = 0.0;
    if (inb) {
        double o = 0.0;
        if (c.invD[i] != 0.0) {
            auto ld = [&](long j) { return vin[j] * sc; };
            o = lc_stencil<double, SYM, false>(c, i, ld);
            if (!SYM) o = 0.5 * (o + lc_stencil<double, false, true>(c, i, ld));
            a0 = vin[i] * sc * o;
        }
        u[i] = o;
    }
    const double s0 = block_sum(a0, lds);
    if (threadIdx.x == 0 && threadIdx.y == 0) part[block_linear_id()] = s0;
}

void lc_lz_apply(const CoarseLevel& C, const double* v, const double* scal, double* u,
                 double* partials, hipStream_t s) {
    if (C.sym)
        hipLaunchKernelGGL((k_lc_lz_apply<true>), lc_grid(C), dim3(kThreads), 0, s,
                           C.view<double>(), v, scal, u, partials);
    else
        hipLaunchKernelGGL((k_lc_lz_apply<false>), lc_grid(C), dim3(kThreads), 0, s,
                           C.view<double>(), v, scal, u, partials);
    HIPCHECK(hipGetLastError());
}

// prev <- w = D^-1 u - alpha_k s_k cur - beta_{k-1} s_{k-1} prev; partials of w.(D w).
__global__ void __launch_bounds__(kThreads) k_lc_lz_update(LCView<double> c,
                                                          const double* __restrict__ u,
                                                          const double* __restrict__ cur,
                                                          double* __restrict__ prev,
                                                          const double* __restrict__ scal,
                                                          double* part) {
    __shared__ double lds[kThreads / kWave];
    const double ac = scal[S_ALPHA] * scal[S_LZ_S], bp = scal[S_LZ_B] * scal[S_LZ_SP];
    LC_PROLOGUE
    double a0 = 0.0;
    if (inb) {
        const double id = c.invD[i];
        if (id != 0.0) {
            const double w = id * u[i] - ac * cur[i] - bp * prev[i];
            prev[i] = w;
            a0 = w * w / id;
        }
    }
    const double s0 = block_sum(a0, lds);
    if (threadIdx.x == 0 && threadIdx.y == 0) part[block_linear_id()] = s0;
}

void lc_lz_update(const CoarseLevel& C, const double* u, const double* cur, double* prev,
                  const double* scal, double* partials, hipStream_t s) {
    hipLaunchKernelGGL(k_lc_lz_update, lc_grid(C), dim3(kThreads), 0, s, C.view<double>(), u,
                       cur, prev, scal, partials);
    HIPCHECK(hipGetLastError());
}

// Chebyshev step with D^-1 (see the level-0 version for the modes).  CHEB_ZERO2 takes
// D^-1 f in xin (written by the restriction that produced f), so that each neighbour
// costs one load.
template <typename T, bool SYM, int MODE>
__global__ void __launch_bounds__(kMThreads) k_lc_cheb(LCView<T> c, LcTile tl,
                                                       const T* __restrict__ f,
                                                       const T* __restrict__ xin,
                                                       const T* __restrict__ din,
                                                       T* __restrict__ xout, T* __restrict__ dout,
                                                       T c1, T c2, T c20) {
    struct R {
        T id, fi, di;
    };
    // CHEB_ZERO1 has no stencil: it marches over f (any valid vector) and ignores ax
    const T* xs = MODE == CHEB_ZERO1 ? f : xin;
    lc_march<T, SYM, false>(
        c, tl, LC_LOAD(xs),
        [&](long i) { return R{c.invD[i], f[i], MODE == CHEB_NEXT ? din[i] : T(0)}; },
        [&](long i, const R& r, T xc, T axs, bool comp) {
            if (!comp) return;
            const T id = r.id;
            T xo = 0, dn = 0;
            if (id != (T)0) {
                const T fi = r.fi;
                if (MODE == CHEB_ZERO1) {
                    xo = c20 * id * fi;
                    dn = xo;
                } else if (MODE == CHEB_ZERO2) {
                    const T ax = c20 * axs;
                    const T x1 = c20 * id * fi;
                    dn = c1 * x1 + c2 * id * (fi - ax);
                    xo = x1 + dn;
                } else {
                    const T rr = id * (fi - axs);
                    dn = (MODE == CHEB_FIRST) ? c20 * rr : c1 * r.di + c2 * rr;
                    xo = xc + dn;
                }
            }
            xout[i] = xo;
            if (dout) dout[i] = dn;
        });
}

// Algorithmic bytes of one coarse-level stencil sweep: slots, 1/diag and `nvec` vectors
// over the level's unknowns, plus the table rows.
static inline long lc_bytes(const CoarseLevel& C, int wsize, int nvec) {
    return C.n_unknowns * (4L + (long)wsize * (1 + nvec)) + C.n_tab * 27L * wsize;
}

template <typename T>
void lc_cheb(const CoarseLevel& C, int mode, const T* f, const T* xin, const T* din, T* xout,
             T* dout, double c1, double c2, double c2_0, hipStream_t s) {
    const int nvec = mode == CHEB_ZERO1 ? 2 : mode == CHEB_NEXT ? 4 : 3;
    KTimer kt_(T_COARSE, s, lc_bytes(C, sizeof(T), nvec + (dout ? 1 : 0)));
    LCView<T> c = C.view<T>();
    const LcTile tl = lc_tiling(C);
    const dim3 g = lc_mgrid(C, tl), b(kWave, kMY);
#define LC_CHEB(SYMV, M)                                                                       \
    klaunch(kt_, true, (k_lc_cheb<T, SYMV, M>), g, b, c, tl, f, xin, din, xout, dout, (T)c1,   \
            (T)c2, (T)c2_0);
#define LC_CHEB_MODES(SYMV)                                 \
    switch (mode) {                                         \
        case CHEB_ZERO1: LC_CHEB(SYMV, CHEB_ZERO1) break;   \
        case CHEB_ZERO2: LC_CHEB(SYMV, CHEB_ZERO2) break;   \
        case CHEB_FIRST: LC_CHEB(SYMV, CHEB_FIRST) break;   \
        default: LC_CHEB(SYMV, CHEB_NEXT) break;            \
    }
    if (C.sym) {
        LC_CHEB_MODES(true)
    } else {
        LC_CHEB_MODES(false)
    }
#undef LC_CHEB_MODES
#undef LC_CHEB
    HIPCHECK(hipGetLastError());
}
template void lc_cheb<double>(const CoarseLevel&, int, const double*, const double*, const double*,
                              double*, double*, double, double, double, hipStream_t);
template void lc_cheb<float>(const CoarseLevel&, int, const float*, const float*, const float*,
                             float*, float*, double, double, double, hipStream_t);

// r = f - A x and (rd non-null) rd = D^-1 r, the restriction's input.
template <typename T, bool SYM>
__global__ void __launch_bounds__(kMThreads) k_lc_residual(LCView<T> c, LcTile tl,
                                                           const T* __restrict__ f,
                                                           const T* __restrict__ xv,
                                                           T* __restrict__ r, T* __restrict__ rd) {
    struct R {
        T id, fi;
    };
    lc_march<T, SYM, false>(c, tl, LC_LOAD(xv), [&](long i) { return R{c.invD[i], f[i]}; },
                            [&](long i, const R& q, T, T ax, bool comp) {
                                if (!comp) return;
                                const T o = q.id != (T)0 ? q.fi - ax : T(0);
                                r[i] = o;
                                if (rd) rd[i] = q.id * o;
                            });
}

template <typename T>
void lc_residual(const CoarseLevel& C, const T* f, const T* x, T* r, T* rd, hipStream_t s) {
    KTimer kt_(T_COARSE, s, lc_bytes(C, sizeof(T), rd ? 4 : 3));
    const LcTile tl = lc_tiling(C);
    if (C.sym)
        klaunch(kt_, true, (k_lc_residual<T, true>), lc_mgrid(C, tl), dim3(kWave, kMY),
                C.view<T>(), tl, f, x, r, rd);
    else
        klaunch(kt_, true, (k_lc_residual<T, false>), lc_mgrid(C, tl), dim3(kWave, kMY),
                C.view<T>(), tl, f, x, r, rd);
    HIPCHECK(hipGetLastError());
}
template void lc_residual<double>(const CoarseLevel&, const double*, const double*, double*,
                                  double*, hipStream_t);
template void lc_residual<float>(const CoarseLevel&, const float*, const float*, float*, float*,
                                 hipStream_t);

// out = D^-1 in on every storage node (0 off the unknowns and on the ghost layer).
template <typename T>
__global__ void __launch_bounds__(256) k_lc_dscale(const T* __restrict__ invD,
                                                   const T* __restrict__ in, T* __restrict__ out,
                                                   long n) {
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < n) out[i] = invD[i] * in[i];
}

template <typename T>
void lc_dscale(const CoarseLevel& C, const T* in, T* out, hipStream_t s) {
    const T* invD;
    if constexpr (sizeof(T) == 8) invD = C.invD64;
    else invD = C.invD32;
    hipLaunchKernelGGL((k_lc_dscale<T>), dim3((unsigned)((C.nstore + 255) / 256)), dim3(256), 0, s,
                       invD, in, out, C.nstore);
    HIPCHECK(hipGetLastError());
}
template void lc_dscale<double>(const CoarseLevel&, const double*, double*, hipStream_t);
template void lc_dscale<float>(const CoarseLevel&, const float*, float*, hipStream_t);

// P^T r with P = (I - w D^-1 A) P_tent in two passes: y = r - w A^T (D^-1 r) on every fine
// node (one thread per node; y overwrites r in place, each thread reading only its own r),
// then fc(I) = sum of y over aggregate I, and (fd non-null) fd = D_c^-1 fc for the coarse
// level's first smoothing step.
template <typename T, bool SYM>
__global__ void __launch_bounds__(kMThreads) k_lc_restrict_y(LCView<T> c, LcTile tl, T* ry,
                                                             const T* __restrict__ rd, T omega) {
    lc_march<T, SYM, true>(c, tl, LC_LOAD(rd), [&](long i) { return ry[i]; },
                           [&](long i, T ri, T, T atr, bool comp) {
                               if (comp) ry[i] = ri - omega * atr;
                           });
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_lc_restrict_sum(LCView<T> f, LCView<T> c,
                                                              const T* __restrict__ yv,
                                                              T* __restrict__ fc,
                                                              T* __restrict__ fd) {
    LC_PROLOGUE
    if (!inb) return;
    T acc = 0;
    for (int dz = 0; dz < 3; ++dz) {
        const int z = 3 * Z + dz;
        if (z >= f.mz) break;
        for (int dy = 0; dy < 3; ++dy) {
            const int y = 3 * Y + dy;
            if (y >= f.my) break;
            const long row = (long)f.sx * (y + 1) + f.sxy * (z + 1) + 1;
            for (int dx = 0; dx < 3; ++dx) {
                const int x = 3 * X + dx;
                if (x < f.mx) acc += yv[row + x];
            }
        }
    }
    fc[i] = acc;
    if (fd) fd[i] = c.invD[i] * acc;
}

template <typename T>
void lc_restrict(const CoarseLevel& F, const CoarseLevel& C, T* r, const T* rd, T* fc, T* fd,
                 double omega, hipStream_t s) {
    KTimer kt_(T_COARSE, s, lc_bytes(F, sizeof(T), 3) +
                                C.n_unknowns * (long)sizeof(T) * (fd ? 3 : 1));
    const LcTile tl = lc_tiling(F);
    if (F.sym)
        klaunch(kt_, false, (k_lc_restrict_y<T, true>), lc_mgrid(F, tl), dim3(kWave, kMY),
                F.view<T>(), tl, r, rd, (T)omega);
    else
        klaunch(kt_, false, (k_lc_restrict_y<T, false>), lc_mgrid(F, tl), dim3(kWave, kMY),
                F.view<T>(), tl, r, rd, (T)omega);
    klaunch(kt_, true, (k_lc_restrict_sum<T>), lc_grid(C), dim3(kThreads), F.view<T>(),
            C.view<T>(), (const T*)r, fc, fd);
    HIPCHECK(hipGetLastError());
}
template void lc_restrict<double>(const CoarseLevel&, const CoarseLevel&, double*, const double*,
                                  double*, double*, double, hipStream_t);
template void lc_restrict<float>(const CoarseLevel&, const CoarseLevel&, float*, const float*,
                                 float*, float*, double, hipStream_t);

// x += P v = P_tent v - w D^-1 A P_tent v on the fine level's unknowns: the stencil runs
// on the field P_tent v, whose value at fine node (x, y, z) is v at its aggregate (floor
// division, so that ghost neighbours (-1) map into the coarse ghost layer).
template <typename T, bool SYM>
__global__ void __launch_bounds__(kMThreads) k_lc_prolong(LCView<T> c, LcTile tl, LCView<T> cc,
                                                          const T* __restrict__ vc,
                                                          T* __restrict__ xv, T omega) {
    struct R {
        T id, x;
    };
    lc_march<T, SYM, false>(
        c, tl,
        [&](long, int xs, int ys, int zs) {  // storage coordinates: logical + 1
            const int ax = (xs + 2) / 3, ay = (ys + 2) / 3, az = (zs + 2) / 3;
            return vc[ax + (long)cc.sx * ay + cc.sxy * az];
        },
        [&](long i) { return R{c.invD[i], xv[i]}; },
        [&](long i, const R& r, T pv, T apv, bool comp) {
            if (comp && r.id != (T)0) xv[i] = r.x + (pv - omega * r.id * apv);
        });
}

template <typename T>
void lc_prolong(const CoarseLevel& F, const CoarseLevel& C, const T* vc, T* x, double omega,
                hipStream_t s) {
    KTimer kt_(T_COARSE, s, lc_bytes(F, sizeof(T), 2) + C.n_unknowns * (long)sizeof(T));
    const LcTile tl = lc_tiling(F);
    if (F.sym)
        klaunch(kt_, true, (k_lc_prolong<T, true>), lc_mgrid(F, tl), dim3(kWave, kMY),
                F.view<T>(), tl, C.view<T>(), vc, x, (T)omega);
    else
        klaunch(kt_, true, (k_lc_prolong<T, false>), lc_mgrid(F, tl), dim3(kWave, kMY),
                F.view<T>(), tl, C.view<T>(), vc, x, (T)omega);
    HIPCHECK(hipGetLastError());
}
template void lc_prolong<double>(const CoarseLevel&, const CoarseLevel&, const double*, double*,
                                 double, hipStream_t);
template void lc_prolong<float>(const CoarseLevel&, const CoarseLevel&, const float*, float*,
                                double, hipStream_t);

// ================================================================ Galerkin product
//
// Column J of A_c = P^T A P with P = (I - w D^-1 A) P_tent, computed on the 9^3 patch of
// fine nodes around aggregate J:  u = P_tent e_J (3^3), v = u - w D^-1 A u (5^3),
// t = A v (7^3), y = t - w A^T D^-1 t (9^3), then A_c(J + c, J) = sum of y over
// aggregate J + c for the 27 neighbouring aggregates c.  The accessor gives the fine
// level's rows (row), transposed rows (rowT), D^-1 and the unknown flag.

struct L0Slot {
    long i;
    bool unk, irr;
    int rank;
};

__device__ inline L0Slot l0_slot(const L0View<double>& v, int x, int y, int z) {
    L0Slot n;
    n.i = x + (long)v.nx * y + v.nxy * z;
    const long seg = ((long)z * v.ny + y) * v.nsegx + (x >> 6);
    const int b = x & 63;
    const uint64_t u = v.unk[seg], r = v.irr[seg];
    n.unk = (u >> b) & 1ull;
    n.irr = (r >> b) & 1ull;
    n.rank = n.irr ? v.base[seg] + __popcll(r & ((1ull << b) - 1ull)) : 0;
    return n;
}

struct AccL0 {
    // k_rap reads the patch's rows through codes computed once per node (kCache)
    static constexpr bool kCache = true;
    L0View<double> v;
    __device__ bool inbox(int x, int y, int z) const {
        return x >= 0 && y >= 0 && z >= 0 && x < v.nx && y < v.ny && z < v.nz;
    }
    // -1: not an unknown (or outside the box), -2: the interior row, else its table slot
    __device__ int code(int x, int y, int z) const {
        if (!inbox(x, y, z)) return -1;
        const L0Slot n = l0_slot(v, x, y, z);
        return !n.unk ? -1 : (n.irr ? n.rank : -2);
    }
    // the rows of rows() from a node's code
    __device__ void rows_code(int c, double* a, double* at, bool* unk) const {
        for (int k = 0; k < 27; ++k) a[k] = at[k] = 0.0;
        *unk = c != -1;
        if (c == -1) return;
        a[13] = at[13] = 1.0;
        for (int d = 0; d < 6; ++d) {
            const int k = dir_to_k(d);
            a[k] = c >= 0 ? v.tcoef(d, c) : v.c[d >> 1];
            at[k] = c >= 0 ? v.tcoefT(d, c) : v.c[d >> 1];
        }
    }
    __device__ double invd_code(int c) const { return c != -1 ? 1.0 : 0.0; }
    // 7-point rows: entries k = 13 and the six direction slots, zero elsewhere
    __device__ void rows(int x, int y, int z, double* a, double* at, bool* unk) const {
        for (int k = 0; k < 27; ++k) a[k] = at[k] = 0.0;
        *unk = false;
        if (!inbox(x, y, z)) return;
        const L0Slot n = l0_slot(v, x, y, z);
        if (!n.unk) return;
        *unk = true;
        a[13] = at[13] = 1.0;
        for (int d = 0; d < 6; ++d) {
            const int k = dir_to_k(d);
            a[k] = n.irr ? v.tcoef(d, n.rank) : v.c[d >> 1];
            at[k] = n.irr ? v.tcoefT(d, n.rank) : v.c[d >> 1];
        }
    }
    __device__ double invd(int x, int y, int z) const {
        if (!inbox(x, y, z)) return 0.0;
        return l0_slot(v, x, y, z).unk ? 1.0 : 0.0;
    }
};

struct AccLC {
    static constexpr bool kCache = false;
    LCView<double> c;
    __device__ int code(int, int, int) const { return 0; }
    __device__ void rows_code(int, double*, double*, bool*) const {}
    __device__ double invd_code(int) const { return 0.0; }
    __device__ bool inbox(int x, int y, int z) const {
        return x >= 0 && y >= 0 && z >= 0 && x < c.mx && y < c.my && z < c.mz;
    }
    __device__ long sidx(int x, int y, int z) const {
        return (x + 1) + (long)c.sx * (y + 1) + c.sxy * (z + 1);
    }
    __device__ void rows(int x, int y, int z, double* a, double* at, bool* unk) const {
        for (int k = 0; k < 27; ++k) a[k] = at[k] = 0.0;
        *unk = false;
        if (!inbox(x, y, z)) return;
        const long i = sidx(x, y, z);
        if (c.invD[i] == 0.0) return;
        *unk = true;
        for (int k = 0; k < 27; ++k) {
            a[k] = lc_full(c, i, k);
            at[k] = c.sym ? a[k] : lc_full(c, i + c.off[k], 26 - k);
        }
    }
    __device__ double invd(int x, int y, int z) const {
        if (!inbox(x, y, z)) return 0.0;
        return c.invD[sidx(x, y, z)];
    }
};

// The 27 output arrays of a Galerkin product, passed by value with the launch.
struct CoefOut {
    double* p[27];
};

template <class Acc>
__global__ void __launch_bounds__(256) k_rap(Acc acc, int fmx, int fmy, int fmz, LCView<double> cc,
                                             CoefOut out, double omega) {
    __shared__ double sv[125], sw[343], sy[729];
    __shared__ int sc[Acc::kCache ? 729 : 1];  // codes of the patch's nodes (Acc::kCache)
    // aggregate of this workgroup.  Workgroups are dealt to the XCDs round-robin; on levels
    // >= 1 (27 fp64 arrays read per patch) the remap gives each XCD a run of consecutive
    // aggregates (neighbours along X, whose patches overlap by two thirds), so that they
    // share its L2: the product from the 1,478,912-unknown level fetched 7.85 GB from memory
    // without it and 1.16 GB with it.  Level 0 (a few MB of masks and table) keeps the
    // plain order, measured as fast or faster there.
    const unsigned b = blockIdx.x, q8 = gridDim.x >> 3;
    const unsigned lb = (!Acc::kCache && b < 8 * q8) ? (b & 7) * q8 + (b >> 3) : b;
    const int X = (int)(lb % (unsigned)cc.mx), Y = (int)((lb / (unsigned)cc.mx) % (unsigned)cc.my),
              Z = (int)(lb / ((unsigned)cc.mx * (unsigned)cc.my));
    const int t = threadIdx.x;
    // patch position p (0..8 per axis) -> fine logical 3J - 3 + p
    const int ox = 3 * X - 3, oy = 3 * Y - 3, oz = 3 * Z - 3;
    double a[27], at[27];
    bool unk;
    // skip empty aggregates
    int has = 0;
    if (t < 27) {
        const int px = 3 + t % 3, py = 3 + (t / 3) % 3, pz = 3 + t / 9;
        acc.rows(ox + px, oy + py, oz + pz, a, at, &unk);
        has = unk ? 1 : 0;
    }
    if (!__syncthreads_or(has)) return;
    // every node the phases below evaluate lies in the 9^3 patch
    if constexpr (Acc::kCache) {
        for (int q = t; q < 729; q += blockDim.x) sc[q] = acc.code(ox + q % 9, oy + (q / 9) % 9, oz + q / 81);
        __syncthreads();
    }
    auto rows_at = [&](int px, int py, int pz, double* ra, double* rat, bool* ru) {
        if constexpr (Acc::kCache)
            acc.rows_code(sc[px + 9 * py + 81 * pz], ra, rat, ru);
        else
            acc.rows(ox + px, oy + py, oz + pz, ra, rat, ru);
    };
    auto invd_at = [&](int px, int py, int pz) {
        if constexpr (Acc::kCache)
            return acc.invd_code(sc[px + 9 * py + 81 * pz]);
        else
            return acc.invd(ox + px, oy + py, oz + pz);
    };

    auto in_block = [](int px, int py, int pz) {
        return px >= 3 && px < 6 && py >= 3 && py < 6 && pz >= 3 && pz < 6;
    };
    // the offsets k (increasing) at which a row can be nonzero: the 7-point stencil on
    // level 0, all 27 on the coarse levels.  Skipped terms are exact zeros, so the sums
    // are those of the full loops.
    auto for_k = [&](auto f) {
        if constexpr (Acc::kCache) {
            constexpr int k7[7] = {4, 10, 12, 13, 14, 16, 22};
#pragma unroll
            for (int j = 0; j < 7; ++j) f(k7[j]);
        } else {
            for (int k = 0; k < 27; ++k) f(k);
        }
    };
    // phase 1: v on [2,7)^3
    for (int q = t; q < 125; q += blockDim.x) {
        const int px = 2 + q % 5, py = 2 + (q / 5) % 5, pz = 2 + q / 25;
        rows_at(px, py, pz, a, at, &unk);
        double s = 0.0;
        for_k([&](int k) {
            const int dx = k % 3 - 1, dy = (k / 3) % 3 - 1, dz = k / 9 - 1;
            if (in_block(px + dx, py + dy, pz + dz)) s += a[k];
        });
        const double u = (unk && in_block(px, py, pz)) ? 1.0 : 0.0;
        sv[q] = u - omega * invd_at(px, py, pz) * s;
    }
    __syncthreads();
    // phase 2: t = A v on [1,8)^3
    for (int q = t; q < 343; q += blockDim.x) {
        const int px = 1 + q % 7, py = 1 + (q / 7) % 7, pz = 1 + q / 49;
        rows_at(px, py, pz, a, at, &unk);
        double s = 0.0;
        for_k([&](int k) {
            const int qx = px + k % 3 - 1 - 2, qy = py + (k / 3) % 3 - 1 - 2, qz = pz + k / 9 - 1 - 2;
            if (qx >= 0 && qx < 5 && qy >= 0 && qy < 5 && qz >= 0 && qz < 5)
                s += a[k] * sv[qx + 5 * qy + 25 * qz];
        });
        sw[q] = s;
    }
    __syncthreads();
    // phase 3: y = t - w A^T D^-1 t on [0,9)^3 (zero at nodes that are not unknowns)
    for (int q = t; q < 729; q += blockDim.x) {
        const int px = q % 9, py = (q / 9) % 9, pz = q / 81;
        rows_at(px, py, pz, a, at, &unk);
        double yv = 0.0;
        if (unk) {
            double s = 0.0;
            for_k([&](int k) {
                const int dx = k % 3 - 1, dy = (k / 3) % 3 - 1, dz = k / 9 - 1;
                const int qx = px + dx - 1, qy = py + dy - 1, qz = pz + dz - 1;
                if (qx >= 0 && qx < 7 && qy >= 0 && qy < 7 && qz >= 0 && qz < 7 && at[k] != 0.0)
                    s += at[k] * invd_at(px + dx, py + dy, pz + dz) * sw[qx + 7 * qy + 49 * qz];
            });
            const bool inw = px >= 1 && px < 8 && py >= 1 && py < 8 && pz >= 1 && pz < 8;
            const double tv = inw ? sw[(px - 1) + 7 * (py - 1) + 49 * (pz - 1)] : 0.0;
            yv = tv - omega * s;
        }
        sy[q] = yv;
    }
    __syncthreads();
    // phase 4: sums over the 27 aggregates J + c
    if (t < 27) {
        const int cx = t % 3 - 1, cy = (t / 3) % 3 - 1, cz = t / 9 - 1;
        const int IX = X + cx, IY = Y + cy, IZ = Z + cz;
        const int kprime = 26 - t;  // offset index of -c
        if (IX >= 0 && IY >= 0 && IZ >= 0 && IX < cc.mx && IY < cc.my && IZ < cc.mz &&
            (!cc.sym || kprime >= 13)) {
            double s = 0.0;
            for (int q = 0; q < 27; ++q) {
                const int px = 3 + 3 * cx + q % 3, py = 3 + 3 * cy + (q / 3) % 3,
                          pz = 3 + 3 * cz + q / 9;
                s += sy[px + 9 * py + 81 * pz];
            }
            const long row = (IX + 1) + (long)cc.sx * (IY + 1) + cc.sxy * (IZ + 1);
            out.p[kprime][row] = s;
        }
    }
    (void)fmx;
    (void)fmy;
    (void)fmz;
}

static CoefOut coef_out(const CoarseLevel& C) {
    CoefOut o;
    for (int k = 0; k < 27; ++k) o.p[k] = C.coef64[k];
    return o;
}

void rap_from_l0(const FineLevel& L, const CoarseLevel& C, double omega, hipStream_t s) {
    AccL0 acc{L.view<double>()};
    const dim3 g((unsigned)((long)C.mx * C.my * C.mz));  // one workgroup per aggregate
    hipLaunchKernelGGL((k_rap<AccL0>), g, dim3(256), 0, s, acc, L.nx, L.ny, L.nz, C.view<double>(),
                       coef_out(C), omega);
    HIPCHECK(hipGetLastError());
}

void rap_from_lc(const CoarseLevel& F, const CoarseLevel& C, double omega, hipStream_t s) {
    AccLC acc{F.view<double>()};
    const dim3 g((unsigned)((long)C.mx * C.my * C.mz));  // one workgroup per aggregate
    hipLaunchKernelGGL((k_rap<AccLC>), g, dim3(256), 0, s, acc, F.mx, F.my, F.mz, C.view<double>(),
                       coef_out(C), omega);
    HIPCHECK(hipGetLastError());
}

// invD = 1/diag at existing coarse nodes (diag != 0); per-block counts of unknowns.
__global__ void k_lc_finish(const double* __restrict__ diag, double* __restrict__ invD, long n,
                            int32_t* cnt) {
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const bool u = t < n && diag[t] != 0.0;
    if (t < n) invD[t] = u ? 1.0 / diag[t] : 0.0;
    const uint64_t bal = __ballot(u);
    if ((threadIdx.x & 63) == 0) cnt[t >> 6] = __popcll(bal);
}

void lc_finish(CoarseLevel& C, int32_t* counts, hipStream_t s) {
    const long nb = (C.nstore + 255) / 256;  // counts: 4 * nb entries
    hipLaunchKernelGGL(k_lc_finish, dim3(nb), dim3(256), 0, s, C.coef64[13], C.invD64, C.nstore,
                       counts);
    HIPCHECK(hipGetLastError());
}

__global__ void k_d2f(const double* a, float* b, long n) {
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t < n) b[t] = (float)a[t];
}

void lc_to_fp32(CoarseLevel& C, hipStream_t s) {
    const long nb = (C.nstore + 255) / 256;
    const long nt = kLcRow * C.tab_cap;
    hipLaunchKernelGGL(k_d2f, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, C.tab64, C.tab32,
                       nt);
    if (C.tabT64) {
        const long ntt = kLcRow * C.tabT_cap;
        hipLaunchKernelGGL(k_d2f, dim3((unsigned)((ntt + 255) / 256)), dim3(256), 0, s, C.tabT64,
                           C.tabT32, ntt);
    }
    hipLaunchKernelGGL(k_d2f, dim3(nb), dim3(256), 0, s, C.invD64, C.invD32, C.nstore);
    HIPCHECK(hipGetLastError());
}

// Compression of a level's operator (after lc_finish).  Pass 1: slot -2 at nodes that are
// not unknowns, -1 where the row equals the reference row `ref` bit for bit (ref < 0:
// none does), -3 where the row equals, bit for bit, the row of the node one plane below
// (which then has a table row of its own or shares one further down), else a new table
// row; per-64 counts of new rows.  Pass 2: table slots of the new rows in storage order,
// and their table rows.  Pass 3: each column, walked up along z, gives its -3 nodes the
// slot of the node below.  A pipe whose cross-section does not change along z repeats
// almost every row from plane to plane, so the table holds a few rows per column of the
// cross-section instead of one per node, and sweeps stream a small, cached table.
__device__ inline bool same_bits(double a, double b) {
    return __double_as_longlong(a) == __double_as_longlong(b);
}

__global__ void k_lc_classify(LCView<double> c, long n, long ref, int32_t* __restrict__ slot,
                              int32_t* __restrict__ cnt) {
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    bool fresh = false;
    if (t < n) {
        int sv = -2;
        if (c.invD[t] != 0.0) {
            bool same = ref >= 0;
            for (int k = 0; k < 27 && same; ++k) same = lc_full(c, t, k) == lc_full(c, ref, k);
            if (same) {
                sv = -1;
            } else {
                // only an unknown below (storage plane >= 1, so every access of its row,
                // including the symmetric storage's neighbour reads, stays in the box)
                bool below = t >= c.sxy && c.invD[t - c.sxy] != 0.0;
                for (int k = 0; k < 27 && below; ++k)
                    below = same_bits(lc_full(c, t, k), lc_full(c, t - c.sxy, k));
                sv = below ? -3 : 0;
                fresh = !below;
            }
        }
        slot[t] = sv;
    }
    const uint64_t bal = __ballot(fresh);
    if ((threadIdx.x & 63) == 0 && t < n) cnt[t >> 6] = __popcll(bal);
}

// Pass 3: nodes marked -3 take the slot of the node one plane below, column by column.
__global__ void k_lc_zshare(int32_t* __restrict__ slot, int sx, int sy, int sz) {
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= (long)sx * sy) return;
    const long sxy = (long)sx * sy;
    for (int z = 1; z < sz; ++z) {
        const long i = t + sxy * z;
        if (slot[i] == -3) slot[i] = slot[i - sxy];
    }
}

__global__ void k_lc_fill(LCView<double> c, long n, const int32_t* __restrict__ base, long cap,
                          int32_t* __restrict__ slot, double* __restrict__ tab) {
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const bool irr = t < n && slot[t] == 0;  // the classification's mark
    const uint64_t bal = __ballot(irr);
    if (!irr) return;
    const int lane = threadIdx.x & 63;
    const int s = base[t >> 6] + __popcll(bal & ((1ull << lane) - 1ull));
    slot[t] = s;
    for (int k = 0; k < 27; ++k) tab[(long)kLcRow * s + k] = lc_full(c, t, k);
    tab[(long)kLcRow * s + 27] = 0.0;
}

// Transpose rows: slot -2 where every coupling is zero (not an unknown), -1 where the node
// and its 26 neighbours all have the interior row, -3 where the transposed row equals the
// one of the node below bit for bit, else a new row (marked 0).
__global__ void k_lc_classifyT(LCView<double> c, long n, int32_t* __restrict__ slotT,
                               int32_t* __restrict__ cnt) {
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    bool fresh = false;
    if (t < n) {
        int sv = -2;
        if (c.invD[t] != 0.0) {
            bool reg = true;
            for (int k = 0; k < 27 && reg; ++k) reg = c.slot[t + c.off[k]] == -1;
            if (reg) {
                sv = -1;
            } else {
                bool below = t >= c.sxy && c.invD[t - c.sxy] != 0.0;
                for (int k = 0; k < 27 && below; ++k)
                    below = same_bits(lc_full(c, t + c.off[k], 26 - k),
                                      lc_full(c, t - c.sxy + c.off[k], 26 - k));
                sv = below ? -3 : 0;
                fresh = !below;
            }
        }
        slotT[t] = sv;
    }
    const uint64_t bal = __ballot(fresh);
    if ((threadIdx.x & 63) == 0 && t < n) cnt[t >> 6] = __popcll(bal);
}

__global__ void k_lc_fillT(LCView<double> c, long n, const int32_t* __restrict__ base, long cap,
                           int32_t* __restrict__ slotT, double* __restrict__ tab) {
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const bool irr = t < n && slotT[t] == 0;  // the classification's mark
    const uint64_t bal = __ballot(irr);
    if (!irr) return;
    const int lane = threadIdx.x & 63;
    const int s = base[t >> 6] + __popcll(bal & ((1ull << lane) - 1ull));
    slotT[t] = s;
    for (int k = 0; k < 27; ++k) tab[(long)kLcRow * s + k] = lc_full(c, t + c.off[k], 26 - k);
    tab[(long)kLcRow * s + 27] = 0.0;
}

__global__ void k_lc_ref_row(LCView<double> c, long ref, double* out) {
    const int k = threadIdx.x;
    if (k < 27) out[k] = lc_full(c, ref, k);
}

void lc_compress(CoarseLevel& C, hipStream_t s) {
    const long n = C.nstore, nw = (n + 63) / 64;
    // reference row: the node at the centre of the box, if it is an unknown
    long ref = (C.mx / 2 + 1) + (long)C.sx * (C.my / 2 + 1) + C.sxy * (C.mz / 2 + 1);
    double dref = 0.0;
    HIPCHECK(hipMemcpyAsync(&dref, C.invD64 + ref, 8, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    if (dref == 0.0) ref = -1;
    if (!C.slot) C.slot = (int32_t*)dmalloc(4 * n);
    int32_t* cnt = (int32_t*)dmalloc(4 * nw);
    int32_t* base = (int32_t*)dmalloc(4 * nw);
    int64_t* tot = (int64_t*)dmalloc(8 * scan_words(nw));
    double* row = (double*)dmalloc(8 * 27);
    try {
        LCView<double> v = C.view<double>();
        hipLaunchKernelGGL(k_lc_classify, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, v, n,
                           ref, C.slot, cnt);
        HIPCHECK(hipGetLastError());
        exclusive_scan(cnt, base, nw, tot, s);
        int64_t nt = 0;
        HIPCHECK(hipMemcpyAsync(&nt, tot, 8, hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
        if (nt > C.tab_cap) {  // (re)allocate; the fp32 copy follows in lc_to_fp32's caller
            dfree(C.tab64);
            dfree(C.tab32);
            C.tab32 = nullptr;
            C.tab_cap = std::max<long>(nt, 1);
            C.tab64 = (double*)dmalloc(8 * kLcRow * C.tab_cap);
        }
        if (!C.tab64) {
            C.tab_cap = 1;
            C.tab64 = (double*)dmalloc(8 * kLcRow);
        }
        C.n_tab = nt;
        hipLaunchKernelGGL(k_lc_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, v, n, base,
                           C.tab_cap, C.slot, C.tab64);
        const dim3 gcol((unsigned)((C.sxy + 255) / 256));
        hipLaunchKernelGGL(k_lc_zshare, gcol, dim3(256), 0, s, C.slot, C.sx, C.sy, C.sz);
        HIPCHECK(hipGetLastError());
        for (int k = 0; k < 27; ++k) C.cst64[k] = 0.0;
        if (ref >= 0) {
            hipLaunchKernelGGL(k_lc_ref_row, dim3(1), dim3(64), 0, s, v, ref, row);
            HIPCHECK(hipGetLastError());
            HIPCHECK(hipMemcpyAsync(C.cst64, row, 8 * 27, hipMemcpyDeviceToHost, s));
        }
        HIPCHECK(hipStreamSynchronize(s));
        if (!C.sym) {
            // the transpose, from the slots just built
            if (!C.slotT) C.slotT = (int32_t*)dmalloc(4 * n);
            v = C.view<double>();
            hipLaunchKernelGGL(k_lc_classifyT, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, v,
                               n, C.slotT, cnt);
            HIPCHECK(hipGetLastError());
            exclusive_scan(cnt, base, nw, tot, s);
            int64_t ntt = 0;
            HIPCHECK(hipMemcpyAsync(&ntt, tot, 8, hipMemcpyDeviceToHost, s));
            HIPCHECK(hipStreamSynchronize(s));
            if (ntt > C.tabT_cap || !C.tabT64) {
                dfree(C.tabT64);
                dfree(C.tabT32);
                C.tabT32 = nullptr;
                C.tabT_cap = std::max<long>(ntt, 1);
                C.tabT64 = (double*)dmalloc(8 * kLcRow * C.tabT_cap);
            }
            C.n_tabT = ntt;
            hipLaunchKernelGGL(k_lc_fillT, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, v, n,
                               base, C.tabT_cap, C.slotT, C.tabT64);
            hipLaunchKernelGGL(k_lc_zshare, gcol, dim3(256), 0, s, C.slotT, C.sx, C.sy, C.sz);
            HIPCHECK(hipGetLastError());
            HIPCHECK(hipStreamSynchronize(s));
        }
    } catch (...) {
        for (void* p : {(void*)cnt, (void*)base, (void*)tot, (void*)row}) dfree(p);
        throw;
    }
    for (void* p : {(void*)cnt, (void*)base, (void*)tot, (void*)row}) dfree(p);
}

// Storage indices of the existing nodes of a coarse level, in increasing order.
__global__ void k_lc_list(const double* __restrict__ invD, long n, const int32_t* base,
                          long* out) {
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const bool u = t < n && invD[t] != 0.0;
    const uint64_t bal = __ballot(u);
    if (u) {
        const int lane = threadIdx.x & 63;
        out[base[t >> 6] + __popcll(bal & ((1ull << lane) - 1ull))] = t;
    }
}

void lc_unknown_list(const CoarseLevel& C, long* out, int32_t* counter, hipStream_t s) {
    // counter: per-64 counts already produced by lc_finish; scan them in place into a copy
    const long nw = (C.nstore + 63) / 64;
    int32_t* base = (int32_t*)dmalloc(sizeof(int32_t) * nw);
    int64_t* tot = (int64_t*)dmalloc(sizeof(int64_t) * scan_words(nw));
    exclusive_scan(counter, base, nw, tot, s);
    hipLaunchKernelGGL(k_lc_list, dim3((C.nstore + 255) / 256), dim3(256), 0, s, C.invD64,
                       C.nstore, base, out);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(s));
    dfree(base);
    dfree(tot);
}

// ================================================================ coarsest level

__global__ void k_fill_cmap(int32_t* cmap, const long* cidx, int nL) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nL) cmap[cidx[t]] = t;
}

void fill_cmap(int32_t* cmap, const long* cidx, int nL, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_cmap, dim3((nL + 255) / 256), dim3(256), 0, s, cmap, cidx, nL);
    HIPCHECK(hipGetLastError());
}

__global__ void k_dense_l0(L0View<double> v, const long* cidx, const int32_t* cmap, int nL,
                           double* A) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nL) return;
    const long b = cidx[i];
    const int x = b % v.nx, y = (b / v.nx) % v.ny, z = b / v.nxy;
    AccL0 acc{v};
    double a[27], at[27];
    bool unk;
    acc.rows(x, y, z, a, at, &unk);
    for (int k = 0; k < 27; ++k) {
        if (a[k] == 0.0) continue;
        const int dx = k % 3 - 1, dy = (k / 3) % 3 - 1, dz = k / 9 - 1;
        const int j = cmap[b + dx + (long)v.nx * dy + v.nxy * dz];
        if (j >= 0) A[(long)i * nL + j] = a[k];
    }
}

__global__ void k_dense_lc(LCView<double> c, const long* cidx, const int32_t* cmap, int nL,
                           double* A) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nL) return;
    const long m = cidx[i];
    for (int k = 0; k < 27; ++k) {
        const double a = lc_full(c, m, k);
        if (a == 0.0) continue;
        const int j = cmap[m + c.off[k]];
        if (j >= 0) A[(long)i * nL + j] = a;
    }
}

void dense_from_l0(const FineLevel& L, const long* cidx, const int32_t* cmap, int nL, double* A,
                   hipStream_t s) {
    hipLaunchKernelGGL(k_dense_l0, dim3((nL + 63) / 64), dim3(64), 0, s, L.view<double>(), cidx,
                       cmap, nL, A);
    HIPCHECK(hipGetLastError());
}

void dense_from_lc(const CoarseLevel& C, const long* cidx, const int32_t* cmap, int nL, double* A,
                   hipStream_t s) {
    hipLaunchKernelGGL(k_dense_lc, dim3((nL + 63) / 64), dim3(64), 0, s, C.view<double>(), cidx,
                       cmap, nL, A);
    HIPCHECK(hipGetLastError());
}

// In-place inversion of the coarsest operator A (row-major n x n, fp64) by Gauss-Jordan
// elimination without pivoting (A is positive definite, or has a positive definite
// symmetric part, so every pivot is positive), taken in blocks of kGjB pivots.  For the
// block K = [k0, k0 + kb), with P = (A_KK)^-1:
//   A_Kj <- P A_Kj (j outside K),  A_ij <- A_ij - A_iK A_Kj (new)  and  A_iK <- -A_iK P
//   (i outside K),  A_KK <- P,
// which is kb single-pivot steps applied at once.  Two launches per block: the first
// inverts A_KK in LDS (every workgroup, the same arithmetic), forms the block row on the
// matrix cores and saves the old block column; the second does the rank-kb update on the
// matrix cores.
constexpr int kGjB = 32;

typedef double gj_d4 __attribute__((ext_vector_type(4)));

// Block step, part 1 (1024 threads).  Every workgroup inverts A_KK in LDS, one thread per
// element of the kGjB x kGjB block and one barrier per pivot (the block is double-buffered:
// pivot p reads buffer p % 2 and writes the other); entries past kb stay zero.  Then:
//  * wavefront w forms the block row P A_Kj for the 16 columns j0 = 256 g + 16 w (outside
//    the block) on the matrix cores, as two 16 x 16 tiles of kGjB / 4 steps each;
//  * rows i = 256 g + t / 4 (outside the block) copy their old block-column entries to C
//    (n x kGjB, 8 per thread, zero past kb);
//  * workgroup 0 stores P (kGjB x kGjB, zero past kb).
// Every global load is issued before the inversion.  Matrix-core operand layouts: see
// k_gjb_update.
__global__ void __launch_bounds__(1024) k_gjb_panel(double* __restrict__ A, int n, int k0, int kb,
                                                    double* __restrict__ Pout,
                                                    double* __restrict__ C) {
    __shared__ double M[2][kGjB][kGjB + 1];
    const int t = threadIdx.x, r = t / kGjB, c = t % kGjB;
    const int lane = t & 63, w = t >> 6, lr = lane & 15, lk = lane >> 4;
    const bool in = r < kb && c < kb;
    M[0][r][c] = in ? A[(long)(k0 + r) * n + k0 + c] : 0.0;
    // block-row operands: column jb of the old block row, rows 4 m + lk
    const int j0 = blockIdx.x * 256 + 16 * w, jb = j0 + lr;
    const bool tile = j0 < n && !(j0 >= k0 && j0 < k0 + kb);  // uniform over the wavefront
    double bo[kGjB / 4];
#pragma unroll
    for (int m = 0; m < kGjB / 4; ++m) {
        const int q = 4 * m + lk;
        bo[m] = (tile && q < kb && jb < n) ? A[(long)(k0 + q) * n + jb] : 0.0;
    }
    // old block column of row ic, entries c8 .. c8 + 7
    const int ic = blockIdx.x * 256 + t / 4, c8 = 8 * (t % 4);
    const bool crow = ic < n && (ic < k0 || ic >= k0 + kb);
    double cv[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) cv[e] = (crow && c8 + e < kb) ? A[(long)ic * n + k0 + c8 + e] : 0.0;
    __syncthreads();
    for (int p = 0; p < kb; ++p) {
        const int b = p & 1;
        const double mpp = M[b][p][p], mpc = M[b][p][c], mrp = M[b][r][p], mrc = M[b][r][c];
        const double piv = 1.0 / mpp;
        const double pc = mpc * piv;  // scaled pivot row (rounded before use)
        double v;
        if (r == p)
            v = (c == p) ? piv : pc;
        else
            v = (c == p) ? -mrp * piv : mrc - mrp * pc;
        M[b ^ 1][r][c] = in ? v : 0.0;
        __syncthreads();
    }
    const int f = kb & 1;  // buffer holding P
    if (tile) {
        gj_d4 d0 = {0.0, 0.0, 0.0, 0.0}, d1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int m = 0; m < kGjB / 4; ++m) {
            d0 = __builtin_amdgcn_mfma_f64_16x16x4f64(M[f][lr][4 * m + lk], bo[m], d0, 0, 0, 0);
            d1 = __builtin_amdgcn_mfma_f64_16x16x4f64(M[f][16 + lr][4 * m + lk], bo[m], d1, 0, 0, 0);
        }
        if (jb < n)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r0 = lk + 4 * v, r1 = 16 + lk + 4 * v;
                if (r0 < kb) A[(long)(k0 + r0) * n + jb] = d0[v];
                if (r1 < kb) A[(long)(k0 + r1) * n + jb] = d1[v];
            }
    }
    if (crow)
#pragma unroll
        for (int e = 0; e < 8; ++e) C[(long)ic * kGjB + c8 + e] = cv[e];
    if (blockIdx.x == 0) Pout[t] = M[f][r][c];
}

// Block step, part 2, on 16 x 16 tiles, one per wavefront (tile rows i0 = 16 blockIdx.y,
// columns j0 = 64 blockIdx.x + 16 w).  K is kGjB-aligned and ends at a multiple of 16 or
// at n, so a tile lies wholly inside or outside the block on each axis.  Outside the
// block row, S = C_iK B_Kj with B_Kj the new block row (P's columns where j is in K) is
// formed by v_mfma_f64_16x16x4_f64 over kGjB / 4 steps of 4 pivots, and A_ij <- A_ij - S
// (A_iK <- -S in the block column).  Inside the block row only A_KK <- P is written (part
// 1 wrote the rest).  Operand layouts of the instruction (lane l, 16 x 4 times 4 x 16):
// A[l % 16][l / 16], B[l / 16][l % 16]; accumulator element v of lane l is
// D[l / 16 + 4 v][l % 16] (rows interleaved by 4 across the lane groups, as measured on
// gfx950).
__global__ void __launch_bounds__(256) k_gjb_update(double* __restrict__ A, int n, int k0, int kb,
                                                    const double* __restrict__ P,
                                                    const double* __restrict__ C) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i0 = 16 * blockIdx.y, j0 = 64 * blockIdx.x + 16 * w;
    if (j0 >= n) return;  // uniform over the wavefront
    const bool rowK = i0 >= k0 && i0 < k0 + kb, colK = j0 >= k0 && j0 < k0 + kb;
    const int lr = lane & 15, lk = lane >> 4;
    if (rowK) {
        if (colK)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = i0 + lk + 4 * v, j = j0 + lr;
                if (i < n && j < n) A[(long)i * n + j] = P[(i - k0) * kGjB + (j - k0)];
            }
        return;
    }
    const int ia = i0 + lr;  // this lane's row of the C operand
    const int jb = j0 + lr;  // this lane's column of the B operand
    double a[kGjB / 4], b[kGjB / 4];
#pragma unroll
    for (int m = 0; m < kGjB / 4; ++m) {
        const int c = 4 * m + lk;
        a[m] = ia < n ? C[(long)ia * kGjB + c] : 0.0;
        if (colK)
            b[m] = P[c * kGjB + (jb - k0)];
        else
            b[m] = (c < kb && jb < n) ? A[(long)(k0 + c) * n + jb] : 0.0;
    }
    double cur[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = i0 + lk + 4 * v;
        cur[v] = (!colK && i < n && jb < n) ? A[(long)i * n + jb] : 0.0;
    }
    gj_d4 s = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int m = 0; m < kGjB / 4; ++m) s = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m], b[m], s, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = i0 + lk + 4 * v;
        if (i < n && jb < n) A[(long)i * n + jb] = cur[v] - s[v];
    }
}

// In-place inverse of the n x n matrix A (row-major, fp64): 2 launches per block of kGjB
// pivots.
void dense_invert(double* A, int n, hipStream_t s) {
    Tmp P(sizeof(double) * kGjB * kGjB), C(sizeof(double) * (size_t)n * kGjB);
    const unsigned gcol = (unsigned)((n + 255) / 256);
    const dim3 gup((unsigned)((n + 63) / 64), (unsigned)((n + 15) / 16));
    for (int k0 = 0; k0 < n; k0 += kGjB) {
        const int kb = std::min(kGjB, n - k0);
        hipLaunchKernelGGL(k_gjb_panel, dim3(gcol), dim3(1024), 0, s, A, n, k0, kb, P.as<double>(),
                           C.as<double>());
        hipLaunchKernelGGL(k_gjb_update, gup, dim3(256), 0, s, A, n, k0, kb,
                           (const double*)P.as<double>(), (const double*)C.as<double>());
    }
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(s));
}

// Gauss-Seidel sweeps on the coarsest level from x = 0 (the iterative coarse level
// solver of Section 3.2), in fp64 with the level's fp64 coefficients.  Unknowns are
// visited colour by colour, colour = parities of the logical coordinates; the 27-point
// stencil never couples two unknowns of one colour, so each colour is updated in parallel
// and the result is the sequential sweep in that order.  One workgroup; the iterate lives
// in LDS (storage size at most kGsMax).
template <typename TF, typename T, bool SYM>
__global__ void __launch_bounds__(1024) k_coarse_gs(LCView<double> c, const TF* __restrict__ f,
                                                    T* __restrict__ x, int sweeps) {
    __shared__ double xs[kGsMax];
    if (c.skip && *c.skip != 0.0) return;  // before any barrier: the whole block returns
    const long n = (long)c.sx * c.sy * (c.mz + 2);
    for (long i = threadIdx.x; i < n; i += blockDim.x) xs[i] = 0.0;
    __syncthreads();
    for (int sw = 0; sw < sweeps; ++sw) {
        for (int col = 0; col < 8; ++col) {
            for (long i = threadIdx.x; i < n; i += blockDim.x) {
                const double id = c.invD[i];
                if (id == 0.0) continue;
                const long X = i % c.sx - 1, Y = (i / c.sx) % c.sy - 1, Z = i / c.sxy - 1;
                if ((int)((X & 1) + 2 * (Y & 1) + 4 * (Z & 1)) != col) continue;
                const double ax = lc_stencil<double, SYM, false>(c, i, [&](long j) { return xs[j]; });
                xs[i] += id * ((double)f[i] - ax);
            }
            __syncthreads();
        }
    }
    for (long i = threadIdx.x; i < n; i += blockDim.x)
        if (c.invD[i] != 0.0) x[i] = (T)xs[i];
}

template <typename TF, typename T>
void coarse_gs(const CoarseLevel& C, const TF* f, T* x, int sweeps, hipStream_t s) {
    KTimer kt_(T_COARSE, s, C.n_unknowns * (long)(8 * ((C.sym ? 14 : 27) + 1) + sizeof(TF) + sizeof(T)));
    if (C.sym)
        klaunch(kt_, true, (k_coarse_gs<TF, T, true>), dim3(1), dim3(1024), C.view<double>(), f, x,
                sweeps);
    else
        klaunch(kt_, true, (k_coarse_gs<TF, T, false>), dim3(1), dim3(1024), C.view<double>(), f,
                x, sweeps);
    HIPCHECK(hipGetLastError());
}
template void coarse_gs<double, double>(const CoarseLevel&, const double*, double*, int, hipStream_t);
template void coarse_gs<float, float>(const CoarseLevel&, const float*, float*, int, hipStream_t);

// x[cidx[i]] = sum_j Ainv[i][j] f[cidx[j]] in fp64; one wavefront per row.
template <typename TF, typename T>
__global__ void __launch_bounds__(256) k_coarse_solve(const double* __restrict__ Ainv,
                                                      const long* __restrict__ cidx, int nL,
                                                      const TF* __restrict__ f, T* __restrict__ x,
                                                      const double* __restrict__ skip) {
    if (skip && *skip != 0.0) return;
    const int row = blockIdx.x * 4 + threadIdx.x / kWave;
    const int lane = threadIdx.x & 63;
    if (row >= nL) return;
    double acc = 0.0;
    for (int j = lane; j < nL; j += kWave) acc += Ainv[(long)row * nL + j] * (double)f[cidx[j]];
    acc = wave_sum(acc);
    if (lane == 0) x[cidx[row]] = (T)acc;
}

template <typename TF, typename T>
void coarse_solve(const double* Ainv, const long* cidx, int nL, const TF* f, T* x, hipStream_t s) {
    KTimer kt_(T_COARSE, s, 8L * nL * nL + nL * (long)(sizeof(TF) + sizeof(T) + 8));
    klaunch(kt_, true, (k_coarse_solve<TF, T>), dim3((nL + 3) / 4), dim3(256), Ainv, cidx, nL, f,
            x, g_vskip);
    HIPCHECK(hipGetLastError());
}
template void coarse_solve<double, double>(const double*, const long*, int, const double*, double*,
                                           hipStream_t);
template void coarse_solve<double, float>(const double*, const long*, int, const double*, float*,
                                          hipStream_t);
template void coarse_solve<float, float>(const double*, const long*, int, const float*, float*,
                                         hipStream_t);

__global__ void k_f2d(const float* a, double* b, long n) {
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t < n) b[t] = (double)a[t];
}

void f2d_copy(const float* a, double* b, long n, hipStream_t s) {
    hipLaunchKernelGGL(k_f2d, dim3((n + 255) / 256), dim3(256), 0, s, a, b, n);
    HIPCHECK(hipGetLastError());
}

}  // namespace saamg
