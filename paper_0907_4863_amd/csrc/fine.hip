// Level-0 (lattice) kernels: operator build, stencils, Chebyshev steps, transfer
// operators to level 1, and the fused fp64 CG vector kernels.
//
// Solve-time kernels use one mapping: every wavefront owns one 64-node x-segment of one
// line and marches along z through `zb` planes.  A block of 4 wavefronts takes 4
// consecutive segments of one line (the whole 256-node line of the large grids; 2 x 2
// or 1 x 4 on narrow boxes), so each plane of a block is one contiguous run of memory.
// Segment masks are wave-uniform (scalar values) and empty segments are skipped.  Along
// z each lane carries its column (z-1, z, z+1) in registers; x-neighbours come from
// adjacent lanes, y-neighbours from L1/L2.  Block numbers are remapped so that the
// blocks dispatched to one XCD form a contiguous z-slab of tiles (the chip hands out
// blocks round-robin over its 8 XCDs, each with its own L2).  Every level-0 work vector
// is zero at the nodes that are not unknowns from allocation on; kernels write only
// unknown nodes, except that in mixed precision the kernels write whole rows (the zero
// written back at the non-unknowns of the rows they store; kFullRows).
#include "march.h"

namespace saamg {

// setup kernels: plain 3-D grid of 64 x 4 blocks, kZBS planes per block
constexpr int kZBS = 4;

static inline dim3 l0_grid(const FineLevel& L) {
    return dim3(L.nsegx, (L.ny + kBlockY - 1) / kBlockY, (L.nz + kZBS - 1) / kZBS);
}

// Level-0 metadata streamed by every stencil launch: segment masks and table slots,
// plus the irregular rows' coefficients.
static inline long l0_meta_bytes(const FineLevel& L, int wsize, bool trans_too) {
    return L.nseg * 20 + L.n_tab * 6L * wsize * (trans_too ? 2 : 1);
}


// Planes per block for the solve-time kernels: long z-marches, but enough blocks to
// fill the chip a few times over.
constexpr long kMinBlocks = 8192;
int l0_choose_zb(int tx, int nsegx, int ny, int nz) {
    const int ty = kMY / tx;
    const long tiles = (long)((nsegx + tx - 1) / tx) * ((ny + ty - 1) / ty);
    int zb = 32;
    while (zb > 2 && tiles * ((nz + zb - 1) / zb) < kMinBlocks) zb /= 2;
    return zb;
}

// 16-byte lanes by default where rows start 16-byte aligned and a line spans more than two
// 64-node segments (shorter lines would leave most lanes of a 256-node span idle).
bool l0_wide_default(int nx) { return nx % 4 == 0 && nx > 128; }

// On a hierarchy with 16-byte lanes every V-cycle kernel, the CG's residual and the CG
// step (its ring form, below) run on them (measured per kernel on the 256 x 256 x 768
// elliptic pipe, one-node against 16-byte lanes, us per launch: fp32 residual 132 -> 107,
// restriction pass 125 -> 89; fp64 residual 282 -> 204, restriction pass 208 -> 141).

long cg_resid_parts(const FineLevel& L) { return L.wide ? l0_wblocks(L, 2) : l0_blocks(L); }
long cg_pq_parts(const FineLevel& L, bool ring, int bytes) {
    return ring ? l0_wblocks(L, cg_dir_lanes(bytes)) : l0_blocks(L);
}
long cg_xr_parts(const FineLevel& L, bool ring, int bytes) {
    return ring ? l0_wblocks(L, cg_xr_lanes(bytes)) : l0_blocks(L);
}
long l0_dot_parts(const FineLevel& L, int bytes) {
    return L.wide ? l0_wblocks(L, dot_lanes(bytes)) : l0_blocks(L);
}

// Planes per block of the kernels on 16-byte lanes: at most 64 / n - 2 (the per-tile word
// preload), else as l0_choose_zb with a lower block target (the wider lanes need fewer
// wavefronts to keep the memory system busy; measured on the 256 x 256 x 768 box, 4 nodes
// per lane: 8 planes 110.1 us, 16 planes 110.0 us, 4 planes 113.3 us per residual).
constexpr long kMinWideBlocks = 2048;
int l0_wide_zb(const FineLevel& L, int n, int planes) {
    const int cap = kWave / n - 2;
    if (planes) return std::min(planes, cap);
    int zb = 1;
    while (2 * zb <= cap) zb *= 2;
    const int nws = (L.nx + kWave * n - 1) / (kWave * n);
    const int tx = nws >= kMY ? kMY : (nws >= 2 ? 2 : 1);
    const long tiles = (long)((nws + tx - 1) / tx) * ((L.ny + kMY / tx - 1) / (kMY / tx));
    while (zb > 2 && tiles * ((L.nz + zb - 1) / zb) < kMinWideBlocks) zb /= 2;
    return zb;
}

long l0_blocks(const FineLevel& L) {
    const int tx = L.tx, ty = kMY / tx;
    const long gx = (L.nsegx + tx - 1) / tx, gy = (L.ny + ty - 1) / ty;
    return gx * gy * ((L.nz + L.zb - 1) / L.zb);
}

static inline dim3 l0_mgrid(const FineLevel& L) { return dim3((unsigned)l0_blocks(L)); }

// Per-lane view of one level-0 node (setup kernels).
struct L0Node {
    long i;       // box index
    bool unk;     // unknown
    bool irr;     // irregular row
    int rank;     // table slot when irregular
};

template <typename T>
__device__ inline L0Node l0_node(const L0View<T>& v, int x, int y, int z) {
    L0Node n;
    n.i = x + (long)v.nx * y + v.nxy * z;
    n.unk = false;
    n.irr = false;
    n.rank = 0;
    if (x < v.nx && y < v.ny) {
        const long seg = ((long)z * v.ny + y) * v.nsegx + (x >> 6);
        const int b = x & 63;
        const uint64_t u = v.unk[seg];
        const uint64_t r = v.irr[seg];
        n.unk = (u >> b) & 1ull;
        n.irr = (r >> b) & 1ull;
        if (n.irr) n.rank = v.base[seg] + __popcll(r & ((1ull << b) - 1ull));
    }
    return n;
}

#define L0_LOOP_BEGIN                                              \
    const int x = blockIdx.x * kWave + threadIdx.x;                \
    const int y = blockIdx.y * kBlockY + threadIdx.y;              \
    const int z0 = blockIdx.z * kZBS;                              \
    const int z1 = min(z0 + kZBS, v.nz);                           \
    for (int z = z0; z < z1; ++z) {                                \
        const L0Node n = l0_node(v, x, y, z);                      \
        const bool inb = x < v.nx && y < v.ny;

#define L0_LOOP_END }

// ---------------------------------------------------------------- solve-time engine

// March over this block's tile.  One wavefront owns one 64-node segment row and walks
// it along z.  For every unknown node the march calls
//   fv = fetch(i, x, y, z, irr, rk)            (loads, issued one plane ahead)
//   body(i, fv, c, ax, x, y, z, irr, rk)       (arithmetic and stores)
// with the box index i, coordinates, irregular flag and table slot, the input value
// c = X(i) and, when STENCIL, ax = (A X)_i (TR: A^T X) of the scaled operator, computed
// in T from the values X returns (X may return a narrower type).  X must be zero at
// nodes that are not unknowns.  The segment words of planes z0-1 .. z1 are fetched up
// front (one plane per lane) and broadcast per step; a row without unknowns in the tile
// exits at once.
//
// The loads of a plane are issued one plane ahead, without waiting on anything of the
// current plane, so the loads of plane z+1 are all in flight while plane z is computed
// and a wavefront waits for one memory round trip per plane.  To keep those loads from
// touching lines the row does not need, a lane outside the span [first, last unknown] of
// its row in that plane reads at the nearest end of the span instead (fetch then sees
// that node's index and coordinates); such values are never used by the lane itself and
// are replaced by zero before they serve as a neighbour's x- or z-neighbour.
// With FULL the body also runs on the lanes of a row with unknowns whose node is in the
// box but not an unknown, with table slot -1, so that a kernel can store every lane of
// the row (zero at those nodes) in one full-width write.
// x-neighbours come from adjacent lanes (the two edge lanes load theirs), z-neighbours
// from registers, y-neighbours from L1/L2; table rows are loaded by the irregular lanes.
template <typename T, typename TX, class FV>
struct PlaneLoads {
    uint64_t u;   // unknown bits of the segment row
    bool irr;
    bool ins1;    // lane inside the row's unknown span in plane z+1
    int rk;
    bool tab;     // the row has irregular nodes: t holds table rows
    long ib;      // box index of lane 0 of the row in this plane (wave-uniform)
    TX nxt, ym, yp, edge;  // X at (x, y, z+1), (x, y-1, z), (x, y+1, z), lane-edge x-neighbour
    T t[6];                // table row of an irregular node
    FV fv;
};

template <typename T, bool STENCIL, bool TR, bool FULL = false, class Load, class Fetch, class Body,
          class End = NoEnd>
__device__ __forceinline__ void l0_march(const L0View<T>& v, Load X, Fetch fetch, Body body,
                                         End end = End{}) {
    using FV = decltype(fetch(Idx{0, 0u}, 0, 0, 0, false, 0));
    using TX = decltype(X(Idx{0, 0u}));
    if (v.skip && *v.skip != 0.0) return;  // wave-uniform: the whole grid returns
    int bx, y, bz;
    l0_tile(v, &bx, &y, &bz);
    const int lane = threadIdx.x;
    bx = __builtin_amdgcn_readfirstlane(bx);
    y = __builtin_amdgcn_readfirstlane(y);
    if (y < 1 || y > v.ny - 2 || bx >= v.nsegx) return;
    const int z0 = max(bz * v.zb, 1), z1 = min(bz * v.zb + v.zb, v.nz - 1);
    if (z0 >= z1) return;
    const long nx = v.nx, nxy = v.nxy;
    const T* tb = TR ? v.tabT : v.tab;
    // words of planes q = z0-1+lane, lane < z1-z0+2 (at most zb+2 <= 34 planes)
    uint64_t wu = 0, wr = 0;
    int wb = 0;
    if (lane < z1 - z0 + 2) {
        const long sg = ((long)(z0 - 1 + lane) * v.ny + y) * v.nsegx + bx;
        wu = v.unk[sg];
        wr = v.irr[sg];
        wb = v.base[sg];
    }
    if (__ballot(wu != 0) == 0) return;
    const int x0 = bx * kWave;
    const long rb = x0 + nx * y;  // box index of lane 0 at plane 0
    const long ib_last = rb + nxy * (z1 - 1);
    const int eo = lane == 0 ? -1 : (lane == kWave - 1 ? 1 : 0);
    // X of this lane in the plane with row base ibq (k = plane - (z0 - 1)), read inside the
    // plane's span
    auto load_x = [&](int k, long ibq) {
        return X(Idx{ibq, (unsigned)span_lane(lane_u64(wu, k), lane)});
    };
    // loads of plane q, whose row base ib = rb + nxy * q the caller carries along
    auto load_plane = [&](int q, long ib) {
        PlaneLoads<T, TX, FV> P;
        P.ib = ib;
        const int k = q - (z0 - 1);
        P.u = lane_u64(wu, k);
        const uint64_t r = lane_u64(wr, k);
        const int lc = span_lane(P.u, lane);
        const bool ins = lc == lane;
        P.ins1 = span_lane(lane_u64(wu, k + 1), lane) == lane;
        P.irr = (r >> lane) & 1ull;
        const int rbase = __builtin_amdgcn_readlane(wb, k);
        const unsigned rofs = __popcll(r & ((1ull << lane) - 1ull));
        P.rk = P.irr ? rbase + (int)rofs : 0;
        P.fv = fetch(Idx{ib, (unsigned)lc}, x0 + lc, y, q, P.irr, P.rk);
        if (STENCIL) {
            P.nxt = load_x(k + 1, ib + nxy);
            P.ym = X(Idx{ib - nx, (unsigned)lc});
            P.yp = X(Idx{ib + nx, (unsigned)lc});
            // the edge lanes' outer x-neighbours (from a base one node lower, so that the
            // offset stays non-negative); only those two lanes load
            P.edge = TX(0);
            if (lane == 0 || lane == kWave - 1)
                P.edge = X(Idx{ib - 1, (unsigned)(lc + 1 + (ins ? eo : 0))});
            // rows with an irregular node: the irregular lanes read their table row
            P.tab = r != 0;
            if (P.tab) {
#pragma unroll
                for (int d = 0; d < 6; ++d) P.t[d] = T(0);
                if (P.irr) load_row6(tb, rbase, rofs, P.t);
            } else {
#pragma unroll
                for (int d = 0; d < 6; ++d) P.t[d] = T(0);
            }
        }
        return P;
    };
    TX zm = TX(0), c = TX(0);
    if (STENCIL) {
        zm = load_x(0, rb + nxy * (z0 - 1));
        c = load_x(1, rb + nxy * z0);
        if (span_lane(lane_u64(wu, 0), lane) != lane) zm = TX(0);
        if (span_lane(lane_u64(wu, 1), lane) != lane) c = TX(0);
    }
    auto settle_plane = [&](const PlaneLoads<T, TX, FV>& P) {
        if (STENCIL) {
            settle(P.nxt);
            settle(P.ym);
            settle(P.yp);
            settle(P.edge);
            settle(P.t);
        }
        settle(P.fv);
    };
    // Arithmetic of plane z from its loads P (only the settling when the plane is past the
    // tile).
    auto step = [&](const PlaneLoads<T, TX, FV>& P, int z) {
        settle_plane(P);
        if (z >= z1) return;
        // X at (x, y, z+1); zero where that plane's span does not reach
        const TX zp = (STENCIL && P.ins1) ? P.nxt : TX(0);
        if (P.u != 0) {
            TX xm = TX(0), xp = TX(0);
            if (STENCIL) {
                xm = wave_shift<true>(c, P.edge);
                xp = wave_shift<false>(c, P.edge);
            }
            const bool unk = (P.u >> lane) & 1ull;
            if (FULL ? (x0 + lane < v.nx) : unk) {
                const Idx i{P.ib, (unsigned)lane};
                const int r = P.rk;
                T ax = T(0);
                if (STENCIL) {
                    if (!P.irr) {
                        ax = T(c) + v.c[0] * (T(xm) + T(xp)) + v.c[1] * (T(P.ym) + T(P.yp)) +
                             v.c[2] * (T(zm) + T(zp));
                    } else {
                        ax = T(c) + P.t[0] * T(xm) + P.t[1] * T(xp) + P.t[2] * T(P.ym) +
                             P.t[3] * T(P.yp) + P.t[4] * T(zm) + P.t[5] * T(zp);
                    }
                }
                body(i, P.fv, T(c), ax, x0 + lane, y, z, P.irr, (FULL && !unk) ? -1 : r);
            }
        }
        if (STENCIL) {
            zm = c;
            c = zp;
        }
        end(z, z == z1 - 1, x0 + lane, y);
    };
    // Two register sets take turns: while one plane is computed the next one's loads are
    // in flight, and no copy between the sets forces an early wait.  Loads past the tile
    // re-read its last plane; the loop has no early exit, so that no path reaches the
    // loop head with a plane's loads unsettled.
    // The row base advances by one plane per step (no per-plane multiply); past the tile it
    // stays at the last plane's.
    long ibz = rb + nxy * z0;
    PlaneLoads<T, TX, FV> pa = load_plane(z0, ibz);
    for (int z = z0; z < z1; z += 2) {
        const long ib1 = ibz + nxy;
        PlaneLoads<T, TX, FV> pb = load_plane(min(z + 1, z1 - 1), ib1 < ib_last ? ib1 : ib_last);
        step(pa, z);
        ibz += 2 * nxy;
        pa = load_plane(min(z + 2, z1 - 1), ibz < ib_last ? ibz : ib_last);
        step(pb, z + 1);
    }
}


// ================================================================ finalisation

__global__ void __launch_bounds__(kFinThreads) k_finalize(const double* __restrict__ part,
                                                          long nblk, int nq, double* scal, int op,
                                                          int dst) {
    __shared__ double lds[kFinThreads / kWave];
    double sums[3] = {0.0, 0.0, 0.0};
    for (int q = 0; q < nq; ++q) {
        double a = 0.0;
        for (long i = threadIdx.x; i < nblk; i += kFinThreads) a += part[q * nblk + i];
        const int tid = threadIdx.x;
        a = wave_sum(a);
        if ((tid & 63) == 0) lds[tid >> 6] = a;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int w = 0; w < kFinThreads / kWave; ++w) s += lds[w];
            sums[q] = s;
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    switch (op) {
        case FIN_STORE:
            for (int q = 0; q < nq; ++q) scal[dst + q] = sums[q];
            break;
        case FIN_ALPHA: {
            // the step is taken only when p.q > 0, r.z > 0 and alpha is finite; dst > 0
            // also records the step length there (a direction ring's slot)
            const double a = scal[S_RHO] / sums[0];
            scal[S_PQ] = sums[0];
            scal[S_ALPHA] = a;
            scal[S_XA] = (sums[0] > 0.0 && scal[S_RHO] > 0.0 && isfinite(a)) ? a : 0.0;
            if (dst > 0) scal[dst] = scal[S_XA];
            break;
        }
        case FIN_RHO_INIT:
            scal[S_RHO] = sums[0];
            scal[S_RHO_PREV] = sums[0];
            scal[S_BETA] = 0.0;
            scal[S_XA] = 0.0;
            break;
        case FIN_XA_CLEAR:
            scal[S_XA] = 0.0;
            break;
        case FIN_RHO:
            scal[S_BETA] = sums[0] / scal[S_RHO];
            scal[S_RHO_PREV] = scal[S_RHO];
            scal[S_RHO] = sums[0];
            break;
        case FIN_LZ_ALPHA:  // alpha_k of the Lanczos recurrence, recorded at scal[dst]
            scal[S_ALPHA] = sums[0];
            scal[dst] = sums[0];
            break;
        case FIN_LZ_BETA: {  // beta_k = ||w||_D; the next vector is w / beta_k
            const double b = sqrt(sums[0]);
            scal[dst] = b;
            scal[S_LZ_SP] = scal[S_LZ_S];
            scal[S_LZ_S] = b > 0.0 ? 1.0 / b : 0.0;
            scal[S_LZ_B] = b;
            break;
        }
        case FIN_NORM:  // first Lanczos vector = start / ||start||_D
            scal[S_LZ_S] = 1.0 / sqrt(sums[0]);
            scal[S_LZ_SP] = 0.0;
            scal[S_LZ_B] = 0.0;
            break;
        case FIN_RESTORE_RHO:  // a step redone from the true residual: its V-cycle runs
            scal[S_RHO] = scal[S_RHO_PREV];
            scal[S_SKIP] = 0.0;
            break;
        case FIN_RR: {
            // ||r||^2, and the skip flag of the V-cycle queued next: set when the
            // recursive residual passes the stopping rule, by the host's own expression
            // (sqrt(r.r) / sqrt(b.b) <= tol, same IEEE operations), or is not finite; the
            // host then stops or recomputes the true residual, and never uses that V-cycle
            const double rr = sums[0];
            scal[S_RR] = rr;
            scal[S_SKIP] = !(sqrt(rr) / sqrt(scal[S_BB]) > scal[S_TOL]) ? 1.0 : 0.0;
            break;
        }
    }
}

__global__ void k_scal_start(double* scal, double tol) {
    scal[S_TOL] = tol;
    scal[S_SKIP] = 0.0;
}

void scal_start(double* scal, double tol, hipStream_t s) {
    hipLaunchKernelGGL(k_scal_start, dim3(1), dim3(1), 0, s, scal, tol);
    HIPCHECK(hipGetLastError());
}

void finalize(const double* partials, long nblk, int nq, double* scal, int op, int dst,
              hipStream_t s) {
    KTimer kt_(T_FINALIZE, s, nblk * 8L * nq);
    klaunch(kt_, true, k_finalize, dim3(1), dim3(kFinThreads), partials, nblk, nq, scal, op, dst);
    HIPCHECK(hipGetLastError());
}

// ================================================================ build

__global__ void k_scatter_nwidx(int32_t* nwidx, const int64_t* nodes, long n) {
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t < n) nwidx[nodes[t]] = (int32_t)t;
}

void l0_scatter_nwidx(int32_t* nwidx, const int64_t* nodes, long n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_scatter_nwidx, dim3((n + 255) / 256), dim3(256), 0, s, nwidx, nodes, n);
    HIPCHECK(hipGetLastError());
}

// Segment masks: unknown bits from the mask.  A row is regular only at an interior point
// (all six neighbours are unknowns, Section 2) whose neighbours all have the interior
// diagonal; every other unknown row (a neighbour outside, a wall fraction s < 1 at the
// node or at a neighbour) is irregular and keeps explicit coefficients, zero toward
// outside neighbours.
__global__ void __launch_bounds__(kThreads) k_build_masks(int nx, int ny, int nz, int nsegx,
                                                          const uint8_t* __restrict__ mask,
                                                          const int32_t* __restrict__ nwidx,
                                                          uint64_t* unk, uint64_t* irr,
                                                          int32_t* cnt_irr, int32_t* cnt_unk) {
    const int x = blockIdx.x * kWave + threadIdx.x;
    const int y = blockIdx.y * kBlockY + threadIdx.y;
    const long nxy = (long)nx * ny;
    for (int z = blockIdx.z * kZBS; z < min(blockIdx.z * kZBS + kZBS, nz); ++z) {
        bool u = false, r = false;
        if (x < nx && y < ny) {
            const long i = x + (long)nx * y + nxy * z;
            u = mask[i] != 0;
            if (u) {
                const bool interior = mask[i - 1] && mask[i + 1] && mask[i - nx] &&
                                      mask[i + nx] && mask[i - nxy] && mask[i + nxy];
                r = !interior || nwidx[i] >= 0 || nwidx[i - 1] >= 0 || nwidx[i + 1] >= 0 ||
                    nwidx[i - nx] >= 0 || nwidx[i + nx] >= 0 || nwidx[i - nxy] >= 0 ||
                    nwidx[i + nxy] >= 0;
            }
        }
        const uint64_t bu = __ballot(u);
        const uint64_t br = __ballot(r);
        if (threadIdx.x == 0 && y < ny) {
            const long seg = ((long)z * ny + y) * nsegx + blockIdx.x;
            unk[seg] = bu;
            irr[seg] = br;
            cnt_irr[seg] = __popcll(br);
            cnt_unk[seg] = __popcll(bu);
        }
    }
}

void l0_build_masks(FineLevel& L, const uint8_t* mask, const int32_t* nwidx, int32_t* cnt_irr,
                    int32_t* cnt_unk, hipStream_t s) {
    hipLaunchKernelGGL(k_build_masks, l0_grid(L), dim3(kWave, kBlockY), 0, s, L.nx, L.ny, L.nz,
                       L.nsegx, mask, nwidx, L.unk, L.irr, cnt_irr, cnt_unk);
    HIPCHECK(hipGetLastError());
}

__global__ void k_mask_diff(const uint64_t* __restrict__ a, const uint64_t* __restrict__ b,
                            const uint64_t* __restrict__ c, const uint64_t* __restrict__ d, long n,
                            int* __restrict__ flag) {
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t < n && (a[t] != b[t] || c[t] != d[t])) *flag = 1;
}

bool l0_same_masks(const FineLevel& L, const uint64_t* unk, const uint64_t* irr, hipStream_t s) {
    Tmp flag(sizeof(int));
    hipLaunchKernelGGL(k_mask_diff, dim3((unsigned)((L.nseg + 255) / 256)), dim3(256), 0, s, L.unk,
                       unk, L.irr, irr, L.nseg, flag.as<int>());
    int h = 1;
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipMemcpyAsync(&h, flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    return h == 0;
}

// Exclusive scan of int32 counts (setup only), in int64.  Tiles of kScanTile counts, one
// per workgroup, 16 consecutive counts per thread: the tiles' sums (k_scan_sums), their
// exclusive scan and the total by one workgroup (k_scan_top), then each tile's scan with
// its offset (k_scan_apply).  One tile: k_scan_apply alone, which also writes the total.
constexpr int kScanT = 256, kScanE = 16;
constexpr long kScanTile = (long)kScanT * kScanE;

long scan_words(long n) { return 1 + std::max(1L, (n + kScanTile - 1) / kScanTile); }

// Sum of the 16 counts of this thread (0 past n).
__device__ inline int64_t scan_thread_sum(const int32_t* in, long n, long i0) {
    int64_t s = 0;
#pragma unroll
    for (int e = 0; e < kScanE; ++e) s += (i0 + e < n) ? in[i0 + e] : 0;
    return s;
}

// Exclusive scan of one value per thread over the workgroup (kScanT threads).
__device__ inline int64_t scan_block_excl(int64_t v, int64_t* lds) {
    const int t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
    for (int d = 1; d < kScanT; d <<= 1) {
        const int64_t a = t >= d ? lds[t - d] : 0;
        __syncthreads();
        lds[t] += a;
        __syncthreads();
    }
    return lds[t] - v;  // inclusive minus own
}

__global__ void __launch_bounds__(kScanT) k_scan_sums(const int32_t* __restrict__ in, long n,
                                                     int64_t* __restrict__ bs) {
    __shared__ int64_t lds[kScanT];
    const long i0 = blockIdx.x * kScanTile + (long)threadIdx.x * kScanE;
    const int64_t v = scan_thread_sum(in, n, i0);
    const int64_t ex = scan_block_excl(v, lds);
    if (threadIdx.x == kScanT - 1) bs[blockIdx.x] = ex + v;
}

// bs[0 .. nb) <- exclusive scan in place; *total <- the sum (one workgroup of 1024).
__global__ void __launch_bounds__(1024) k_scan_top(int64_t* bs, long nb, int64_t* total) {
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const long chunk = (nb + 1023) / 1024;
    const long a = t * chunk, b = min(nb, a + chunk);
    int64_t s = 0;
    for (long i = a; i < b; ++i) s += bs[i];
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        int64_t acc = 0;
        for (int k = 0; k < 1024; ++k) {
            const int64_t v = part[k];
            part[k] = acc;
            acc += v;
        }
        *total = acc;
    }
    __syncthreads();
    int64_t acc = part[t];
    for (long i = a; i < b; ++i) {
        const int64_t v = bs[i];
        bs[i] = acc;
        acc += v;
    }
}

// out[i] = (tile offset) + (counts before i in the tile); bs == nullptr: one tile, offset 0,
// and *total = its sum.
__global__ void __launch_bounds__(kScanT) k_scan_apply(const int32_t* __restrict__ in, long n,
                                                      const int64_t* __restrict__ bs,
                                                      int32_t* __restrict__ out, int64_t* total) {
    __shared__ int64_t lds[kScanT];
    const long i0 = blockIdx.x * kScanTile + (long)threadIdx.x * kScanE;
    int32_t c[kScanE];
    int64_t v = 0;
#pragma unroll
    for (int e = 0; e < kScanE; ++e) {
        c[e] = (i0 + e < n) ? in[i0 + e] : 0;
        v += c[e];
    }
    const int64_t ex = scan_block_excl(v, lds);
    if (!bs && total && threadIdx.x == kScanT - 1) *total = ex + v;
    if (!out) return;
    int64_t acc = (bs ? bs[blockIdx.x] : 0) + ex;
#pragma unroll
    for (int e = 0; e < kScanE; ++e) {
        if (i0 + e < n) out[i0 + e] = (int32_t)acc;
        acc += c[e];
    }
}

void exclusive_scan(const int32_t* in, int32_t* out, long n, int64_t* total, hipStream_t s) {
    const long nb = std::max(1L, (n + kScanTile - 1) / kScanTile);
    if (nb == 1) {
        hipLaunchKernelGGL(k_scan_apply, dim3(1), dim3(kScanT), 0, s, in, n,
                           (const int64_t*)nullptr, out, total);
    } else {
        int64_t* bs = total + 1;
        hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nb), dim3(kScanT), 0, s, in, n, bs);
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, bs, nb, total);
        if (out)
            hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kScanT), 0, s, in, n,
                               (const int64_t*)bs, out, (int64_t*)nullptr);
    }
    HIPCHECK(hipGetLastError());
}

struct RowRule {
    double sigma;   // D^-1/2 of the row
    double f[3];    // factor of the off-diagonal toward the inside neighbour, per axis
};

// Per-axis contribution of the wall rules (Section 2): diagonal in units of 1/h^2 and
// the factor of the remaining off-diagonal.  Outside neighbours are substituted by
// constant (u' = 0), linear (u' = (1-1/s) u) or quadratic extrapolation
// (u' = 2(s-1)/s u - (s-1)/(s+1) u'' ; both sides out: u' and u'' from s and t).
__device__ inline void axis_rule(int variant, bool in_m, bool in_p, double s, double t,
                                 double* diag, double* f) {
    if (in_m && in_p) {
        *diag = 2.0;
        *f = 1.0;
        return;
    }
    if (variant == SAAMG_VARIANT_LIN) {
        *diag = (in_m ? 1.0 : 1.0 / s) + (in_p ? 1.0 : 1.0 / t);
        *f = 1.0;
    } else if (variant == SAAMG_VARIANT_QUAD) {
        if (!in_m && !in_p) {
            *diag = 2.0 / (s * t);
            *f = 1.0;
        } else if (!in_m) {
            *diag = 2.0 / s;
            *f = 2.0 / (s + 1.0);
        } else {
            *diag = 2.0 / t;
            *f = 2.0 / (t + 1.0);
        }
    } else {
        *diag = 2.0;
        *f = 1.0;
    }
}

// Rule of the row at box index i.  Rows without a near-wall entry have the interior
// stencil.  On a domain with open ends (rob = 2 h_z / d > 0) the unknowns of planes 1
// and nz-2 are end-plane rows: their outside z-neighbour is u(x'') - (2 h_z / d) u(x)
// (eq. inlet), and the whole row is halved, which keeps the constant and linear rules
// symmetric.
__device__ inline RowRule row_rule(long i, const uint8_t* mask, const int32_t* nwidx,
                                   const double* nwfrac, int variant, double sigma0,
                                   const double ih2[3], const long step[3], int nz, double rob) {
    RowRule r;
    const int k = nwidx[i];
    if (k < 0) {
        r.sigma = sigma0;
        r.f[0] = r.f[1] = r.f[2] = 1.0;
        return r;
    }
    const long zp = i / step[2];
    const bool end = rob > 0.0 && (zp == 1 || zp == nz - 2);
    double D = 0.0;
    for (int a = 0; a < 3; ++a) {
        const bool in_m = mask[i - step[a]] != 0;
        const bool in_p = mask[i + step[a]] != 0;
        double dg, f;
        if (a == 2 && end) {
            dg = 2.0 + rob;
            f = 2.0;
        } else {
            axis_rule(variant, in_m, in_p, nwfrac[6L * k + 2 * a], nwfrac[6L * k + 2 * a + 1], &dg,
                      &f);
        }
        D += dg * ih2[a];
        r.f[a] = f;
    }
    if (end) {
        D *= 0.5;
        for (int a = 0; a < 3; ++a) r.f[a] *= 0.5;
    }
    r.sigma = 1.0 / sqrt(D);
    return r;
}

// Scaled coupling of row `row` to column `col` along axis a (both unknowns).
__device__ inline double scaled_off(const RowRule& row, const RowRule& col, int a,
                                    const double ih2[3]) {
    return -(row.sigma * (row.f[a] * ih2[a])) * col.sigma;
}

__global__ void __launch_bounds__(kThreads) k_build_table(
    L0View<double> v, const uint8_t* __restrict__ mask, const int32_t* __restrict__ nwidx,
    const double* __restrict__ nwfrac, int variant, double sigma0, double ihx2, double ihy2,
    double ihz2, double rob, long n_irr, double* tab, float* tab32, double* sigma) {
    const double ih2[3] = {ihx2, ihy2, ihz2};
    const long step[3] = {1, (long)v.nx, v.nxy};
    L0_LOOP_BEGIN
    if (inb) {
        if (!n.unk) {
            sigma[n.i] = 0.0;
        } else {
            const RowRule me =
                row_rule(n.i, mask, nwidx, nwfrac, variant, sigma0, ih2, step, v.nz, rob);
            sigma[n.i] = me.sigma;
            if (n.irr) {
                for (int d = 0; d < 6; ++d) {
                    const int a = d >> 1;
                    const long j = n.i + ((d & 1) ? step[a] : -step[a]);
                    double fw = 0.0, bw = 0.0;
                    if (mask[j]) {
                        const RowRule nb =
                            row_rule(j, mask, nwidx, nwfrac, variant, sigma0, ih2, step, v.nz, rob);
                        fw = scaled_off(me, nb, a, ih2);
                        bw = scaled_off(nb, me, a, ih2);
                    }
                    tab[8 * n.rank + d] = fw;
                    tab[8 * (n_irr + n.rank) + d] = bw;
                    tab32[8 * n.rank + d] = (float)fw;
                    tab32[8 * (n_irr + n.rank) + d] = (float)bw;
                }
                for (int d = 6; d < 8; ++d) {  // padding
                    tab[8 * n.rank + d] = 0.0;
                    tab[8 * (n_irr + n.rank) + d] = 0.0;
                    tab32[8 * n.rank + d] = 0.0f;
                    tab32[8 * (n_irr + n.rank) + d] = 0.0f;
                }
            }
        }
    }
    L0_LOOP_END
}

void l0_build_table(FineLevel& L, const uint8_t* mask, const int32_t* nwidx, const double* nwfrac,
                    int variant, double sigma0, double* tab64, float* tab32, hipStream_t s) {
    L0View<double> v = L.view<double>();
    v.base = L.base_full;
    hipLaunchKernelGGL(k_build_table, l0_grid(L), dim3(kWave, kBlockY), 0, s, v, mask, nwidx,
                       nwfrac, variant, sigma0, 1.0 / (L.h[0] * L.h[0]), 1.0 / (L.h[1] * L.h[1]),
                       1.0 / (L.h[2] * L.h[2]), L.robin_d > 0.0 ? 2.0 * L.h[2] / L.robin_d : 0.0,
                       L.n_irr, tab64, tab32, L.sigma);
    HIPCHECK(hipGetLastError());
}

// ---- de-duplication of the table along z
//
// A line (y, z) repeats the line below it when each of its segments has the irregular mask
// of the segment one plane below and its table rows (operator and transpose, fp64, bit for
// bit) equal theirs in order.  Such a line's segments take the slots of the rows below, so
// a pipe of constant cross-section stores the rows of a few planes only, and a z-march
// reading the same slots on consecutive planes can keep the rows it has.  The rows of a
// line stay consecutive, as the kernels on 16-byte lanes need.

// One wavefront per line (line = z ny + y): its irregular rows (keep = 0 when it repeats
// the line below) and the repeat flag.
__global__ void __launch_bounds__(kThreads) k_l0_line_info(L0View<double> v,
                                                           const int32_t* __restrict__ bfull,
                                                           const double* __restrict__ full,
                                                           long n_irr, int32_t* keep,
                                                           int32_t* same) {
    const long line = (long)blockIdx.x * kBlockY + threadIdx.y;
    if (line >= (long)v.ny * v.nz) return;
    const int lane = threadIdx.x;
    const long z = line / v.ny;
    const long s0 = line * v.nsegx, sb = s0 - (long)v.ny * v.nsegx;  // this line, line below
    int cnt = 0;
    bool diff = z < 1;
    for (int sx = lane; sx < v.nsegx; sx += kWave) {
        const uint64_t r = v.irr[s0 + sx];
        cnt += (int)__popcll(r);
        if (z >= 1 && r != v.irr[sb + sx]) diff = true;
    }
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) cnt += __shfl_xor(cnt, o);
    bool rep = __ballot(diff) == 0;
    if (rep && cnt > 0) {
        const long r0 = bfull[s0], r1 = bfull[sb];
        bool d2 = false;
        for (long k = lane; k < 8L * cnt; k += kWave) {
            d2 |= __double_as_longlong(full[8 * r0 + k]) != __double_as_longlong(full[8 * r1 + k]);
            d2 |= __double_as_longlong(full[8 * (n_irr + r0) + k]) !=
                  __double_as_longlong(full[8 * (n_irr + r1) + k]);
        }
        rep = __ballot(d2) == 0;
    }
    if (lane == 0) {
        keep[line] = rep ? 0 : cnt;
        same[line] = rep;
    }
}

// Slot of each line's first row: the compacted offset of the last line at or below it
// (same y) that does not repeat.  One thread per y.
__global__ void __launch_bounds__(256) k_l0_line_src(int ny, int nz, const int32_t* __restrict__ same,
                                                     const int32_t* __restrict__ off,
                                                     int32_t* __restrict__ nb) {
    const int y = blockIdx.x * blockDim.x + threadIdx.x;
    if (y >= ny) return;
    int m = 0;
#pragma unroll 8
    for (int z = 0; z < nz; ++z) {
        const long line = (long)z * ny + y;
        m = same[line] ? m : off[line];
        nb[line] = m;
    }
}

// base of every segment: its line's first slot plus its offset inside the line.
__global__ void __launch_bounds__(256) k_l0_seg_base(long nseg, int nsegx,
                                                     const int32_t* __restrict__ bfull,
                                                     const int32_t* __restrict__ nb,
                                                     int32_t* __restrict__ base) {
    const long sg = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (sg >= nseg) return;
    const long line = sg / nsegx;
    base[sg] = nb[line] + (bfull[sg] - bfull[line * nsegx]);
}

// Rows of the lines that do not repeat, to their compacted slots (one wavefront per line).
__global__ void __launch_bounds__(kThreads) k_l0_line_copy(long nlines, int nsegx, const int32_t* __restrict__ bfull,
                                                           const int32_t* __restrict__ keep,
                                                           const int32_t* __restrict__ off,
                                                           long n_irr, long n_tab,
                                                           const double* __restrict__ f64,
                                                           const float* __restrict__ f32,
                                                           double* __restrict__ t64,
                                                           float* __restrict__ t32) {
    const long line = (long)blockIdx.x * kBlockY + threadIdx.y;
    if (line >= nlines) return;
    const int cnt = keep[line];
    if (cnt == 0) return;
    const long src = bfull[line * nsegx], dst = off[line];
    for (long k = threadIdx.x; k < 8L * cnt; k += kWave) {
        t64[8 * dst + k] = f64[8 * src + k];
        t64[8 * (n_tab + dst) + k] = f64[8 * (n_irr + src) + k];
        t32[8 * dst + k] = f32[8 * src + k];
        t32[8 * (n_tab + dst) + k] = f32[8 * (n_irr + src) + k];
    }
}

void l0_dedup_table(FineLevel& L, const double* full64, const float* full32, hipStream_t s) {
    const long nlines = (long)L.ny * L.nz;
    Tmp keep(4 * nlines), same(4 * nlines), off(4 * nlines), nb(4 * nlines),
        tot(8 * scan_words(nlines));
    const dim3 gl((unsigned)((nlines + kBlockY - 1) / kBlockY)), bl(kWave, kBlockY);
    hipLaunchKernelGGL(k_l0_line_info, gl, bl, 0, s, L.view<double>(), (const int32_t*)L.base_full,
                       full64, L.n_irr, keep.as<int32_t>(), same.as<int32_t>());
    exclusive_scan(keep.as<int32_t>(), off.as<int32_t>(), nlines, tot.as<int64_t>(), s);
    hipLaunchKernelGGL(k_l0_line_src, dim3((unsigned)((L.ny + 255) / 256)), dim3(256), 0, s, L.ny,
                       L.nz, (const int32_t*)same.as<int32_t>(), (const int32_t*)off.as<int32_t>(),
                       nb.as<int32_t>());
    hipLaunchKernelGGL(k_l0_seg_base, dim3((unsigned)((L.nseg + 255) / 256)), dim3(256), 0, s,
                       L.nseg, L.nsegx, (const int32_t*)L.base_full, (const int32_t*)nb.as<int32_t>(),
                       L.base);
    int64_t n_tab = 0;
    HIPCHECK(hipMemcpyAsync(&n_tab, tot.p, 8, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    HIPCHECK(hipGetLastError());
    dfree(L.tab64);
    dfree(L.tab32);
    L.tab64 = nullptr;
    L.tab32 = nullptr;
    L.n_tab = n_tab;
    L.tab64 = (double*)dmalloc(8 * 16 * std::max<long>(n_tab, 1));
    L.tab32 = (float*)dmalloc(4 * 16 * std::max<long>(n_tab, 1));
    hipLaunchKernelGGL(k_l0_line_copy, gl, bl, 0, s, nlines, L.nsegx, (const int32_t*)L.base_full,
                       (const int32_t*)keep.as<int32_t>(), (const int32_t*)off.as<int32_t>(),
                       L.n_irr, (long)n_tab, full64, full32, L.tab64, L.tab32);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(s));
}

__global__ void __launch_bounds__(kThreads) k_unknown_list(L0View<double> v, const int32_t* ucnt_base,
                                                           long* out) {
    L0_LOOP_BEGIN
    if (inb && n.unk) {
        const long seg = ((long)z * v.ny + y) * v.nsegx + (x >> 6);
        const uint64_t u = v.unk[seg];
        const int b = x & 63;
        out[ucnt_base[seg] + __popcll(u & ((1ull << b) - 1ull))] = n.i;
    }
    L0_LOOP_END
}

void l0_unknown_list(const FineLevel& L, long* out, hipStream_t s) {
    // rank of unknowns by segment: scan the per-segment unknown counts
    Tmp t_cnt(sizeof(int32_t) * L.nseg), t_base(sizeof(int32_t) * L.nseg),
        t_tot(sizeof(int64_t) * scan_words(L.nseg));
    int32_t* cnt = t_cnt.as<int32_t>();
    int32_t* base = t_base.as<int32_t>();
    int64_t* tot = t_tot.as<int64_t>();
    std::vector<uint64_t> hu(L.nseg);
    HIPCHECK(hipMemcpyAsync(hu.data(), L.unk, sizeof(uint64_t) * L.nseg, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    std::vector<int32_t> hc(L.nseg);
    for (long i = 0; i < L.nseg; ++i) hc[i] = __builtin_popcountll(hu[i]);
    HIPCHECK(hipMemcpyAsync(cnt, hc.data(), sizeof(int32_t) * L.nseg, hipMemcpyHostToDevice, s));
    exclusive_scan(cnt, base, L.nseg, tot, s);
    hipLaunchKernelGGL(k_unknown_list, l0_grid(L), dim3(kWave, kBlockY), 0, s, L.view<double>(),
                       base, out);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(s));
}

// ================================================================ operators

// y = A x (or A^T x) on every box node (zero where not an unknown).
template <typename T, bool TR>
__global__ void __launch_bounds__(kMThreads) k_l0_apply(L0View<T> v, const T* __restrict__ xv,
                                                       T* __restrict__ yv) {
    l0_march<T, true, TR>(v, [&](Idx j) { return at(xv, j); }, NOFETCH,
                          [&](Idx i, NoVals, T, T ax, int, int, int, bool, int) { at(yv, i) = ax; });
}

template <typename T>
void l0_apply(const FineLevel& L, bool trans, const T* x, T* y, hipStream_t s) {
    L0View<T> v = L.view<T>();
    HIPCHECK(hipMemsetAsync(y, 0, sizeof(T) * L.nbox, s));
    if (L.wide) {
        w_apply<T>(L, trans, x, y, s);
        return;
    }
    if (trans)
        hipLaunchKernelGGL((k_l0_apply<T, true>), l0_mgrid(L), dim3(kWave, kMY), 0, s, v, x, y);
    else
        hipLaunchKernelGGL((k_l0_apply<T, false>), l0_mgrid(L), dim3(kWave, kMY), 0, s, v, x, y);
    HIPCHECK(hipGetLastError());
}
template void l0_apply<double>(const FineLevel&, bool, const double*, double*, hipStream_t);
template void l0_apply<float>(const FineLevel&, bool, const float*, float*, hipStream_t);

// Lanczos estimate of the top of the spectrum (D = I on the scaled level 0).  Each
// vector v_k is stored unnormalised as s_k * buf with s_k in scal[S_LZ_S].

// v = start vector at the unknowns; partials of v.v.
__global__ void __launch_bounds__(kMThreads) k_l0_lz_start(L0View<double> v, double* w,
                                                          double* part) {
    __shared__ double lds[kMThreads / kWave];
    double a0 = 0.0;
    l0_march<double, false, false>(v, [&](long) { return 0.0; }, NOFETCH,
                                   [&](Idx i, NoVals, double, double, int, int, int, bool, int) {
                                       const double sv = start_value(i);
                                       at(w, i) = sv;
                                       a0 += sv * sv;
                                   });
    const double s0 = block_sum(a0, lds);
    if (threadIdx.x == 0 && threadIdx.y == 0) part[blockIdx.x] = s0;
}

void l0_lz_start(const FineLevel& L, double* v, double* partials, hipStream_t s) {
    hipLaunchKernelGGL(k_l0_lz_start, l0_mgrid(L), dim3(kWave, kMY), 0, s, L.view<double>(), v,
                       partials);
    HIPCHECK(hipGetLastError());
}

// u = S q with q = vin * scal[S_LZ_S] and S the symmetric part (A + A^T)/2; partials of q.u.
// Regular rows have equal row and column (their neighbours carry the interior
// stencil), so only irregular rows add the transposed table.
template <bool SYM>
__global__ void __launch_bounds__(kMThreads) k_l0_lz_apply(L0View<double> v,
                                                          const double* __restrict__ vin,
                                                          const double* __restrict__ scal,
                                                          double* __restrict__ u, double* part) {
    __shared__ double lds[kMThreads / kWave];
    const double sc = scal[S_LZ_S];
    const long nx = v.nx, nxy = v.nxy;
    double a0 = 0.0;
    l0_march<double, true, false>(
        v, [&](Idx j) { return at(vin, j); }, NOFETCH,
        [&](Idx i, NoVals, double qr, double aqr, int, int, int, bool irr, int r) {
            const double q = sc * qr, aq = sc * aqr;
            double o = aq;
            if (!SYM && irr) {
                double t[6];
                load_row6(v.tabT, (long)r, 0u, t);
                const double at = q + sc * (t[0] * vin[i - 1] + t[1] * vin[i + 1] +
                                            t[2] * vin[i - nx] + t[3] * vin[i + nx] +
                                            t[4] * vin[i - nxy] + t[5] * vin[i + nxy]);
                o = 0.5 * (aq + at);
            }
            at(u, i) = o;
            a0 += q * o;
        });
    const double s0 = block_sum(a0, lds);
    if (threadIdx.x == 0 && threadIdx.y == 0) part[blockIdx.x] = s0;
}

void l0_lz_apply(const FineLevel& L, bool sym, const double* v, const double* scal, double* u,
                 double* partials, hipStream_t s) {
    if (sym)
        hipLaunchKernelGGL(k_l0_lz_apply<true>, l0_mgrid(L), dim3(kWave, kMY), 0, s,
                           L.view<double>(), v, scal, u, partials);
    else
        hipLaunchKernelGGL(k_l0_lz_apply<false>, l0_mgrid(L), dim3(kWave, kMY), 0, s,
                           L.view<double>(), v, scal, u, partials);
    HIPCHECK(hipGetLastError());
}

// prev <- w = u - alpha_k s_k cur - beta_{k-1} s_{k-1} prev; partials of w.w.
__global__ void __launch_bounds__(kMThreads) k_l0_lz_update(L0View<double> v,
                                                           const double* __restrict__ u,
                                                           const double* __restrict__ cur,
                                                           double* __restrict__ prev,
                                                           const double* __restrict__ scal,
                                                           double* part) {
    __shared__ double lds[kMThreads / kWave];
    const double ac = scal[S_ALPHA] * scal[S_LZ_S], bp = scal[S_LZ_B] * scal[S_LZ_SP];
    double a0 = 0.0;
    l0_march<double, false, false>(v, [&](long) { return 0.0; }, NOFETCH,
                                   [&](Idx i, NoVals, double, double, int, int, int, bool, int) {
                                       const double w = at(u, i) - ac * at(cur, i) - bp * at(prev, i);
                                       at(prev, i) = w;
                                       a0 += w * w;
                                   });
    const double s0 = block_sum(a0, lds);
    if (threadIdx.x == 0 && threadIdx.y == 0) part[blockIdx.x] = s0;
}

void l0_lz_update(const FineLevel& L, const double* u, const double* cur, double* prev,
                  const double* scal, double* partials, hipStream_t s) {
    hipLaunchKernelGGL(k_l0_lz_update, l0_mgrid(L), dim3(kWave, kMY), 0, s, L.view<double>(), u,
                       cur, prev, scal, partials);
    HIPCHECK(hipGetLastError());
}

// One Chebyshev step on level 0 (D = I).  Modes:
//   ZERO1: x1 = c2_0 f                                   (degree-1 zero-guess smoother)
//   ZERO2: x1 = c2_0 f on the fly; r1 = f - A x1; d1 = c1 x1 + c2 r1; x2 = x1 + d1
//   FIRST: r = f - A xin; d = c2_0 r; xout = xin + d
//   NEXT : r = f - A xin; d = c1 din + c2 r; xout = xin + d
//   NEXT_X: as NEXT with the previous iterate in din: d = c1 (xin - din) + c2 r, so that
//           the step before it need not store its direction
// Optional partial sums of fdot . xout (the PCG's r . z when this is the last step); with
// fdot NULL the dot is taken with f itself (promoted to fp64).
template <typename TF, typename T, int MODE, bool DOT>
__global__ void __launch_bounds__(kMThreads) k_l0_cheb(L0View<T> v, const TF* __restrict__ f,
                                                      const T* __restrict__ xin,
                                                      const T* __restrict__ din, T* __restrict__ xout,
                                                      T* __restrict__ dout, T c1, T c2, T c20,
                                                      const double* __restrict__ fdot, double* part) {
    __shared__ double lds[kMThreads / kWave];
    double acc = 0.0;
    auto fetch = [&](Idx i, int, int, int, bool, int) {
        Vals<T, 2> a;
        a.v[0] = (MODE == CHEB_FIRST || MODE == CHEB_NEXT || MODE == CHEB_NEXT_X ||
                  MODE == CHEB_ZERO1)
                     ? (T)ntl(f, i)
                     : T(0);
        a.v[1] = (MODE == CHEB_NEXT || MODE == CHEB_NEXT_X) ? ntl(din, i) : T(0);
        Vals<double, 1> b;
        b.v[0] = (DOT && fdot) ? ntl(fdot, i) : 0.0;
        struct R {
            Vals<T, 2> a;
            Vals<double, 1> b;
        };
        return R{a, b};
    };
    auto body = [&](Idx i, auto fv, T cv, T ax, int, int, int, bool, int rk) {
        const bool u = rk >= 0;  // false only on the extra lanes of a full-row store
        const T fi = fv.a.v[0];
        T xo, dn;
        if (MODE == CHEB_ZERO1) {
            xo = c20 * fi;
            dn = xo;
        } else if (MODE == CHEB_ZERO2) {  // cv = f_i, ax = (A f)_i
            const T x1 = c20 * cv;
            dn = c1 * x1 + c2 * (cv - c20 * ax);
            xo = x1 + dn;
        } else {
            const T r = fi - ax;
            const T dprev = (MODE == CHEB_NEXT_X) ? cv - fv.a.v[1] : fv.a.v[1];
            dn = (MODE == CHEB_FIRST) ? c20 * r : c1 * dprev + c2 * r;
            xo = cv + dn;
        }
        nts(xout, i, u ? xo : T(0));
        if (dout) nts(dout, i, u ? dn : T(0));
        if (DOT && u) acc += (fdot ? fv.b.v[0] : (double)fi) * (double)xo;
    };
    if (MODE == CHEB_ZERO1)
        l0_march<T, false, false>(v, [&](long) { return T(0); }, fetch, body);
    else if (MODE == CHEB_ZERO2)
        l0_march<T, true, false, kFullRows<T>>(v, [&](Idx j) { return (T)at(f, j); }, fetch, body);
    else
        l0_march<T, true, false, kFullRows<T>>(v, [&](Idx j) { return at(xin, j); }, fetch, body);
    if (DOT) {
        double sb = block_sum(acc, lds);
        if (threadIdx.x == 0 && threadIdx.y == 0) part[blockIdx.x] = sb;
    }
}

template <typename TF, typename T>
void l0_cheb(const FineLevel& L, int mode, const TF* f, const T* xin, const T* din, T* xout,
             T* dout, double c1, double c2, double c2_0, const double* fdot, double* dot,
             hipStream_t s) {
    const long wf = sizeof(TF), w = sizeof(T), n = L.n_unknowns;
    const long vec = (mode == CHEB_ZERO1 || mode == CHEB_ZERO2) ? wf + w
                     : (mode == CHEB_FIRST) ? wf + 2 * w : wf + 3 * w;
    KTimer kt_(T_L0_CHEB, s, n * (vec + (dout ? w : 0) + (dot && fdot ? 8 : 0)) + l0_meta_bytes(L, w, false));
    if constexpr (std::is_same_v<TF, T>) {
        if (L.wide) {
            w_cheb<T>(L, mode, f, xin, din, xout, dout, c1, c2, c2_0, fdot, dot, kt_);
            return;
        }
    }
    L0View<T> v = L.view<T>();
    dim3 g = l0_mgrid(L), b(kWave, kMY);
#define CHEB_LAUNCH(M)                                                                         \
    if (dot)                                                                                   \
        klaunch(kt_, true, (k_l0_cheb<TF, T, M, true>), g, b, v, f, xin, din, xout, dout,      \
                (T)c1, (T)c2, (T)c2_0, fdot, dot);                                             \
    else                                                                                       \
        klaunch(kt_, true, (k_l0_cheb<TF, T, M, false>), g, b, v, f, xin, din, xout, dout,     \
                (T)c1, (T)c2, (T)c2_0, fdot, dot);
    switch (mode) {
        case CHEB_ZERO1: CHEB_LAUNCH(CHEB_ZERO1) break;
        case CHEB_ZERO2: CHEB_LAUNCH(CHEB_ZERO2) break;
        case CHEB_FIRST: CHEB_LAUNCH(CHEB_FIRST) break;
        case CHEB_NEXT_X: CHEB_LAUNCH(CHEB_NEXT_X) break;
        default: CHEB_LAUNCH(CHEB_NEXT) break;
    }
#undef CHEB_LAUNCH
    HIPCHECK(hipGetLastError());
}
template void l0_cheb<double, double>(const FineLevel&, int, const double*, const double*,
                                      const double*, double*, double*, double, double, double,
                                      const double*, double*, hipStream_t);
template void l0_cheb<float, float>(const FineLevel&, int, const float*, const float*,
                                    const float*, float*, float*, double, double, double,
                                    const double*, double*, hipStream_t);

template <typename TF, typename T>
__global__ void __launch_bounds__(kMThreads) k_l0_residual(L0View<T> v, const TF* __restrict__ f,
                                                          const T* __restrict__ xv,
                                                          T* __restrict__ r) {
    l0_march<T, true, false, kFullRows<T>>(
        v, [&](Idx j) { return at(xv, j); },
        [&](Idx i, int, int, int, bool, int) { return Vals<T, 1>{{(T)ntl(f, i)}}; },
        [&](Idx i, Vals<T, 1> fv, T, T ax, int, int, int, bool, int rk) {
            nts(r, i, rk >= 0 ? fv.v[0] - ax : T(0));
        });
}

template <typename TF, typename T>
void l0_residual(const FineLevel& L, const TF* f, const T* x, T* r, hipStream_t s) {
    KTimer kt_(T_L0_RESID, s, L.n_unknowns * (long)(sizeof(TF) + 2 * sizeof(T)) +
                                 l0_meta_bytes(L, sizeof(T), false));
    if constexpr (std::is_same_v<TF, T>) {
        if (L.wide) {
            w_residual<T>(L, f, x, r, kt_);
            return;
        }
    }
    klaunch(kt_, true, (k_l0_residual<TF, T>), l0_mgrid(L), dim3(kWave, kMY), L.view<T>(), f, x,
            r);
    HIPCHECK(hipGetLastError());
}
template void l0_residual<double, double>(const FineLevel&, const double*, const double*,
                                          double*, hipStream_t);
template void l0_residual<float, float>(const FineLevel&, const float*, const float*, float*,
                                        hipStream_t);

// Restriction to level 1, P^T r with P = (I - w A) P_tent (D = I at level 0), in two
// passes.  Pass 1 forms y = r - w A^T r on every fine unknown and sums each lane's column
// over the three planes of an aggregate (the z-slabs start at multiples of 3), writing one
// value per (x, y, aggregate plane) into yz; pass 2 sums yz over the aggregate's 3 x 3
// (x, y) nodes.  Entries of yz that no unknown reaches stay 0 from allocation on.
template <typename T>
__global__ void __launch_bounds__(kMThreads) k_l0_restrict_y(L0View<T> v, const T* __restrict__ r,
                                                            T* __restrict__ yz, T omega) {
    T acc = T(0);
    l0_march<T, true, true>(
        v, [&](Idx j) { return at(r, j); }, NOFETCH,
        [&](Idx, NoVals, T ri, T atr, int, int, int, bool, int) { acc += ri - omega * atr; },
        [&](int z, bool last, int x, int y) {
            if (z % 3 == 2 || last) {
                if (x < v.nx) yz[x + (long)v.nx * y + v.nxy * (z / 3)] = acc;
                acc = T(0);
            }
        });
}

template <typename T>
__global__ void __launch_bounds__(256) k_l0_restrict_sum(int nx, int ny, int nz, LCView<T> c,
                                                         const T* __restrict__ yv,
                                                         T* __restrict__ fc, T* __restrict__ fd) {
    if (c.skip && *c.skip != 0.0) return;
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= (long)c.mx * c.my) return;
    const int X = (int)(t % c.mx), Y = (int)(t / c.mx), Z = blockIdx.y;
    const long nxy = (long)nx * ny;
    T acc = 0;
    for (int dy = 0; dy < 3; ++dy) {
        const int y = 3 * Y + dy;
        if (y >= ny) break;
        const long row = (long)nx * y + nxy * Z;
        for (int dx = 0; dx < 3; ++dx) {
            const int x = 3 * X + dx;
            if (x < nx) acc += yv[row + x];
        }
    }
    const long i = (X + 1) + (long)c.sx * (Y + 1) + c.sxy * (Z + 1);
    fc[i] = acc;
    if (fd) fd[i] = c.invD[i] * acc;
}

// The second pass over x-folded sums (one value per aggregate x, y and layer): the 3 y-rows.
template <typename T>
__global__ void __launch_bounds__(256) k_l0_restrict_sum3(int nx, int ny, int nz, LCView<T> c,
                                                          const T* __restrict__ yv,
                                                          T* __restrict__ fc, T* __restrict__ fd) {
    if (c.skip && *c.skip != 0.0) return;
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= (long)c.mx * c.my) return;
    const int X = (int)(t % c.mx), Y = (int)(t / c.mx), Z = blockIdx.y;
    const long mxq = (nx + 2) / 3;
    T acc = 0;
    for (int dy = 0; dy < 3; ++dy) {
        const int y = 3 * Y + dy;
        if (y >= ny) break;
        acc += yv[X + mxq * y + mxq * ny * Z];
    }
    const long i = (X + 1) + (long)c.sx * (Y + 1) + c.sxy * (Z + 1);
    fc[i] = acc;
    if (fd) fd[i] = c.invD[i] * acc;
}

template <typename T>
void l0_restrict(const FineLevel& L, const CoarseLevel& C, const T* r, T* y, T* fc, T* fd,
                 double omega, hipStream_t s) {
    KTimer kt_(T_L0_RESTRICT, s, (L.n_unknowns * 5 / 3 + C.n_unknowns * (fd ? 3 : 1)) *
                                        (long)sizeof(T) + l0_meta_bytes(L, sizeof(T), true));
    bool folded = false;
    if (L.wide) {
        folded = w_restrict_y<T>(L, r, y, omega, kt_);
    } else {
        // z-slabs of a multiple of 3 planes, so that no aggregate plane is split between tiles
        L0View<T> v = L.view<T>();
        v.zb = std::max(3, L.zb / 3 * 3);
        const long blocks = (long)v.gx * v.gy * ((L.nz + v.zb - 1) / v.zb);
        klaunch(kt_, false, (k_l0_restrict_y<T>), dim3((unsigned)blocks), dim3(kWave, kMY), v, r,
                y, (T)omega);
    }
    dim3 g((unsigned)(((long)C.mx * C.my + 255) / 256), C.mz);
    if (folded)
        klaunch(kt_, true, (k_l0_restrict_sum3<T>), g, dim3(256), L.nx, L.ny, L.nz, C.view<T>(),
                (const T*)y, fc, fd);
    else
        klaunch(kt_, true, (k_l0_restrict_sum<T>), g, dim3(256), L.nx, L.ny, L.nz, C.view<T>(),
                (const T*)y, fc, fd);
    HIPCHECK(hipGetLastError());
}
template void l0_restrict<double>(const FineLevel&, const CoarseLevel&, const double*, double*,
                                  double*, double*, double, hipStream_t);
template void l0_restrict<float>(const FineLevel&, const CoarseLevel&, const float*, float*, float*,
                                 float*, double, hipStream_t);

// Prolongation from level 1: x += P v = P_tent v - w A (P_tent v).  A node's aggregate
// is (x/3, y/3, z/3); a neighbour's differs by one coarse step exactly when the node sits
// on the corresponding face of its 3^3 block.
template <typename T>
__global__ void __launch_bounds__(kMThreads) k_l0_prolong(L0View<T> v, LCView<T> c,
                                                         const T* __restrict__ vc,
                                                         T* __restrict__ xv, T omega) {
    // the coarse values of the node's aggregate and of the neighbours' aggregates, the
    // current x, and (irregular nodes) the row's table coefficients, all issued a plane
    // ahead.  The three planes of an aggregate layer share the node's own, x- and
    // y-neighbour aggregates: those five values are loaded on the layer's first plane in
    // the tile and kept, and only the z-neighbour on a face plane is loaded per plane.
    // They are taken at the lane's own node (x clamped to the box), not at the
    // span-clamped node the other loads use, so that they hold for every plane.
    struct R {
        Vals<T, 8> f;
        Vals<T, 6> t;
    };
    int cqz = -1;
    T c0 = T(0), cxm = T(0), cxp = T(0), cym = T(0), cyp = T(0);
    auto fetch = [&](Idx i, int xs, int y, int z, bool irr, int rk) {
        const int x = min(xs - (int)i.o + (int)threadIdx.x, v.nx - 1);
        const int qx = x / 3, qy = y / 3, qz = z / 3;
        const long a = (qx + 1) + (long)c.sx * (qy + 1) + c.sxy * (qz + 1);
        if (qz != cqz) {  // wave-uniform
            cqz = qz;
            c0 = vc[a];
            cxm = vc[a - (x - 3 * qx == 0)];
            cxp = vc[a + (x - 3 * qx == 2)];
            cym = vc[a - (y - 3 * qy == 0 ? c.sx : 0)];
            cyp = vc[a + (y - 3 * qy == 2 ? c.sx : 0)];
        }
        const int zr = z - 3 * qz;
        R r;
        r.f.v[0] = c0;
        r.f.v[1] = cxm;
        r.f.v[2] = cxp;
        r.f.v[3] = cym;
        r.f.v[4] = cyp;
        r.f.v[5] = zr == 0 ? vc[a - c.sxy] : c0;
        r.f.v[6] = zr == 2 ? vc[a + c.sxy] : c0;
        r.f.v[7] = ntl(xv, i);
#pragma unroll
        for (int d = 0; d < 6; ++d) r.t.v[d] = T(0);
        if (irr) load_row6(v.tab, (long)rk, 0u, r.t.v);
        return r;
    };
    l0_march<T, false, false, kFullRows<T>>(v, [&](long) { return T(0); }, fetch,
                              [&](Idx i, R r, T, T, int, int, int, bool irrow, int rk) {
        const Vals<T, 8>& f = r.f;
        T apv;
        if (!irrow) {
            apv = f.v[0] + v.c[0] * (f.v[1] + f.v[2]) + v.c[1] * (f.v[3] + f.v[4]) +
                  v.c[2] * (f.v[5] + f.v[6]);
        } else {
            apv = f.v[0] + r.t.v[0] * f.v[1] + r.t.v[1] * f.v[2] + r.t.v[2] * f.v[3] +
                  r.t.v[3] * f.v[4] + r.t.v[4] * f.v[5] + r.t.v[5] * f.v[6];
        }
        nts(xv, i, rk >= 0 ? f.v[7] + (f.v[0] - omega * apv) : T(0));
    });
}

template <typename T>
void l0_prolong(const FineLevel& L, const CoarseLevel& C, const T* vc, T* x, double omega,
                hipStream_t s) {
    KTimer kt_(T_L0_PROLONG, s, (2 * L.n_unknowns + C.n_unknowns) * (long)sizeof(T) +
                                   l0_meta_bytes(L, sizeof(T), false));
    if (L.wide) {
        w_prolong<T>(L, C, vc, x, omega, kt_);
        return;
    }
    klaunch(kt_, true, (k_l0_prolong<T>), l0_mgrid(L), dim3(kWave, kMY), L.view<T>(), C.view<T>(),
            vc, x, (T)omega);
    HIPCHECK(hipGetLastError());
}
template void l0_prolong<double>(const FineLevel&, const CoarseLevel&, const double*, double*,
                                 double, hipStream_t);
template void l0_prolong<float>(const FineLevel&, const CoarseLevel&, const float*, float*,
                                double, hipStream_t);

// ================================================================ CG (fp64)

__global__ void __launch_bounds__(kMThreads) k_cg_init(L0View<double> v, const double* __restrict__ sigma,
                                                      const double* __restrict__ b,
                                                      const double* __restrict__ x0,
                                                      double* __restrict__ bs, double* __restrict__ xv) {
    l0_march<double, false, false>(
        v, [&](long) { return 0.0; },
        [&](Idx i, int, int, int, bool, int) {
            return Vals<double, 3>{{ntl(sigma, i), ntl(b, i), x0 ? ntl(x0, i) : 0.0}};
        },
        [&](Idx i, Vals<double, 3> f, double, double, int, int, int z, bool, int) {
            // end-plane rows of open ends are halved, and so is their right-hand side
            const double rho = (z == 1 || z == v.nz - 2) ? v.rho_end : 1.0;
            nts(bs, i, f.v[0] * rho * f.v[1]);
            nts(xv, i, x0 ? f.v[2] / f.v[0] : 0.0);
        });
}

void cg_init(const FineLevel& L, const double* b, const double* x0, double* bs, double* x,
             hipStream_t s) {
    hipLaunchKernelGGL(k_cg_init, l0_mgrid(L), dim3(kWave, kMY), 0, s, L.view<double>(),
                       L.sigma, b, x0, bs, x);
    HIPCHECK(hipGetLastError());
}

// r = bs - A x; partials of r.r and bs.bs.  ZX: x = 0 (a start without an initial guess),
// so r = bs and the march reads no stencil operand.
template <bool ZX>
__global__ void __launch_bounds__(kMThreads) k_cg_resid(L0View<double> v, const double* __restrict__ bs,
                                                       const double* __restrict__ xv,
                                                       double* __restrict__ r, double* part,
                                                       float* __restrict__ r32) {
    __shared__ double lds[kMThreads / kWave];
    double a0 = 0.0, a1 = 0.0;
    l0_march<double, !ZX, false>(
        v, [&](Idx j) { return ZX ? 0.0 : at(xv, j); },
        [&](Idx i, int, int, int, bool, int) { return Vals<double, 1>{{ntl(bs, i)}}; },
        [&](Idx i, Vals<double, 1> f, double, double ax, int, int, int, bool, int) {
            const double bi = f.v[0];
            const double o = ZX ? bi : bi - ax;
            nts(r, i, o);
            if (r32) nts(r32, i, (float)o);
            a0 += o * o;
            a1 += bi * bi;
        });
    const long bid = blockIdx.x, nb = gridDim.x;
    double s0 = block_sum(a0, lds), s1 = block_sum(a1, lds);
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        part[bid] = s0;
        part[nb + bid] = s1;
    }
}

// x == nullptr: x = 0.
void cg_resid(const FineLevel& L, const double* bs, const double* x, double* r, double* partials,
              float* r32, hipStream_t s) {
    if (L.wide) {
        w_cg_resid(L, bs, x, r, partials, r32, s);
        return;
    }
    if (x)
        hipLaunchKernelGGL(k_cg_resid<false>, l0_mgrid(L), dim3(kWave, kMY), 0, s,
                           L.view<double>(), bs, x, r, partials, r32);
    else
        hipLaunchKernelGGL(k_cg_resid<true>, l0_mgrid(L), dim3(kWave, kMY), 0, s,
                           L.view<double>(), bs, (const double*)nullptr, r, partials, r32);
    HIPCHECK(hipGetLastError());
}

// Direction update with the product by A carried along (fp64 direction):  p <- z + beta p and
// q <- A z + beta q, which equals A p_new because q held A p_old.  Partials of p . q.  The
// previous step's x += alpha p, deferred to here, is applied with the old p as it is read.
// (Forming p_new at every stencil node from z and the old p instead, and q = A p_new, moves
// 8 bytes less per unknown but needs twice the stencil loads: measured slower on the
// 256 x 256 x 768 ellipse, 454 -> 488 us.)
template <typename TZ>
__global__ void __launch_bounds__(kMThreads) k_cg_pq(L0View<double> v, const TZ* __restrict__ zv,
                                                    double* __restrict__ xv,
                                                    double* __restrict__ p, double* __restrict__ q,
                                                    const double* __restrict__ scal, double* part) {
    __shared__ double lds[kMThreads / kWave];
    const double beta = scal[S_BETA];
    const double xa = scal[S_XA];
    double acc = 0.0;
    l0_march<double, true, false, kFullRows<TZ>>(
        v, [&](Idx j) { return at(zv, j); },
        [&](Idx i, int, int, int, bool, int) {
            return Vals<double, 3>{{at(p, i), at(q, i), at(xv, i)}};
        },
        [&](Idx i, Vals<double, 3> f, double zi, double az, int, int, int, bool, int rk) {
            const bool u = rk >= 0;
            const double pi = u ? zi + beta * f.v[0] : 0.0;
            const double qi = u ? az + beta * f.v[1] : 0.0;
            nts(xv, i, u ? f.v[2] + xa * f.v[0] : 0.0);
            nts(p, i, pi);
            nts(q, i, qi);
            acc += pi * qi;
        });
    double sb = block_sum(acc, lds);
    if (threadIdx.x == 0 && threadIdx.y == 0) part[blockIdx.x] = sb;
}

// On 16-byte-lane hierarchies the CG step keeps its directions in a ring, in the working
// precision, and no q = A p vector:
//   pn = z + beta p (rounded to the working precision); partials of pn . A pn   (k_w_cg_pdir)
//   r -= alpha A p, A p in fp64 from the stored direction                       (k_w_cg_xr)
//   x += alpha_j p_j for the ring's directions, when it is full or x is read    (k_cg_xring)
// x += alpha p and r -= alpha A p use the same stored p and alpha, so the recursive
// residual follows the true one in fp64 arithmetic whatever the rounding of alpha (whose
// product pn . A pn mixed precision forms with the fp32 operator); rounding p to fp32 only
// perturbs the conjugacy of the directions, at the level of the fp32 preconditioned
// residual z it is formed from.  Per unknown and step, mixed precision: 12 + 24 bytes plus
// (16 + 4 k) / k for a ring of k (40 with k = 16) against 80 for the fused q-recursion with
// its r update; fp64: 24 + 24 + (16 + 8 k) / k (57) against 80.  On one-node lanes, which
// serve the small boxes where each launch's latency counts more than bytes, the fused
// form stays.
bool cg_ring(const FineLevel& L) { return L.wide; }

template <typename TZ>
void cg_pq(const FineLevel& L, const TZ* z, double* x, double* p, double* q, const double* scal,
           double* partials, hipStream_t s) {
    KTimer kt_(T_CG_PQ, s, L.n_unknowns * (long)(sizeof(TZ) + 48) + l0_meta_bytes(L, 8, false));
    klaunch(kt_, true, (k_cg_pq<TZ>), l0_mgrid(L), dim3(kWave, kMY), L.view<double>(), z, x, p, q,
            scal, partials);
    HIPCHECK(hipGetLastError());
}
template void cg_pq<double>(const FineLevel&, const double*, double*, double*, double*,
                            const double*, double*, hipStream_t);
template void cg_pq<float>(const FineLevel&, const float*, double*, double*, double*,
                           const double*, double*, hipStream_t);

template <class E>
void cg_pdir(const FineLevel& L, const E* z, const E* p, E* pn, const double* scal,
             double* partials, hipStream_t s) {
    // z, p read; pn written
    KTimer kt_(T_CG_PQ, s, L.n_unknowns * 3L * (long)sizeof(E) + l0_meta_bytes(L, 8, false));
    if (!cg_ring(L)) throw ApiError{SAAMG_INVALID_ARG, "the ring form of the CG step needs 16-byte lanes"};
    w_cg_pdir<E>(L, z, p, pn, scal, partials, kt_);
}
template void cg_pdir<float>(const FineLevel&, const float*, const float*, float*, const double*,
                             double*, hipStream_t);
template void cg_pdir<double>(const FineLevel&, const double*, const double*, double*,
                              const double*, double*, hipStream_t);

template <class E>
void cg_xring(const FineLevel& L, double* x, const E* ring, const double* scal,
              const RingSlots& rs, hipStream_t s) {
    // x 8 read and written, one direction per pending step
    KTimer kt_(T_CG_X, s, L.n_unknowns * (16L + (long)sizeof(E) * rs.m));
    if (rs.m < 1 || rs.m > kCgRing || L.nbox % 4 != 0)
        throw ApiError{SAAMG_INVALID_ARG, "ring flush: 1..kCgRing directions, a box of 4-node lanes"};
    w_cg_xring<E>(L, x, ring, scal, rs, kt_);
}
template void cg_xring<float>(const FineLevel&, double*, const float*, const double*,
                              const RingSlots&, hipStream_t);
template void cg_xring<double>(const FineLevel&, double*, const double*, const double*,
                               const RingSlots&, hipStream_t);

template <class E>
void cg_xr_dir(const FineLevel& L, const E* p, double* r, float* r32, const double* scal,
               double* partials, hipStream_t s) {
    // p, r 8 read; r 8 (and r32 4) written
    KTimer kt_(T_CG_XR, s, L.n_unknowns * (16L + (long)sizeof(E) + (r32 ? 4 : 0)) +
                               l0_meta_bytes(L, 8, false));
    if (!cg_ring(L)) throw ApiError{SAAMG_INVALID_ARG, "the ring form of the CG step needs 16-byte lanes"};
    w_cg_xr<E>(L, p, r, r32, scal, partials, kt_);
}
template void cg_xr_dir<float>(const FineLevel&, const float*, double*, float*, const double*,
                               double*, hipStream_t);
template void cg_xr_dir<double>(const FineLevel&, const double*, double*, float*, const double*,
                                double*, hipStream_t);

// r -= alpha q (alpha = S_XA) and partials of r.r; r untouched when the step broke down
// (S_XA = 0).  x receives alpha p later (the next k_cg_pq or k_cg_xflush).  With the fp32
// copy (mixed precision) it stores whole rows (FULL).
template <bool FULL>
__global__ void __launch_bounds__(kMThreads) k_cg_xr(L0View<double> v, double* __restrict__ r,
                                                    const double* __restrict__ q,
                                                    const double* __restrict__ scal, double* part,
                                                    float* __restrict__ r32) {
    __shared__ double lds[kMThreads / kWave];
    const double alpha = scal[S_XA];
    const bool ok = alpha != 0.0;
    double acc = 0.0;
    l0_march<double, false, false, FULL>(
        v, [&](Idx) { return 0.0; },
        [&](Idx i, int, int, int, bool, int) { return Vals<double, 2>{{ntl(r, i), ntl(q, i)}}; },
        [&](Idx i, Vals<double, 2> f, double, double, int, int, int, bool, int rk) {
            const bool u = rk >= 0;
            double ri = u ? f.v[0] : 0.0;
            if (ok) {
                ri = u ? ri - alpha * f.v[1] : 0.0;
                nts(r, i, ri);
                if (r32) nts(r32, i, (float)ri);
            }
            acc += ri * ri;
        });
    double sb = block_sum(acc, lds);
    if (threadIdx.x == 0 && threadIdx.y == 0) part[blockIdx.x] = sb;
}

void cg_xr(const FineLevel& L, double* r, const double* q, const double* scal, double* partials,
           float* r32, hipStream_t s) {
    KTimer kt_(T_CG_XR, s, L.n_unknowns * (24L + (r32 ? 4 : 0)));
    if (r32)
        klaunch(kt_, true, k_cg_xr<true>, l0_mgrid(L), dim3(kWave, kMY), L.view<double>(), r, q,
                scal, partials, r32);
    else
        klaunch(kt_, true, k_cg_xr<false>, l0_mgrid(L), dim3(kWave, kMY), L.view<double>(), r, q,
                scal, partials, r32);
    HIPCHECK(hipGetLastError());
}

template <typename TP>
__global__ void __launch_bounds__(kMThreads) k_cg_xflush(L0View<double> v, double* __restrict__ xv,
                                                        const TP* __restrict__ p,
                                                        const double* __restrict__ scal) {
    const double xa = scal[S_XA];
    l0_march<double, false, false>(
        v, [&](Idx) { return 0.0; },
        [&](Idx i, int, int, int, bool, int) {
            return Vals<double, 2>{{at(xv, i), (double)at(p, i)}};
        },
        [&](Idx i, Vals<double, 2> f, double, double, int, int, int, bool, int) {
            at(xv, i) = f.v[0] + xa * f.v[1];
        });
}

template <typename TP>
void cg_xflush(const FineLevel& L, double* x, const TP* p, const double* scal, hipStream_t s) {
    hipLaunchKernelGGL((k_cg_xflush<TP>), l0_mgrid(L), dim3(kWave, kMY), 0, s, L.view<double>(), x,
                       p, scal);
    HIPCHECK(hipGetLastError());
}
template void cg_xflush<double>(const FineLevel&, double*, const double*, const double*,
                                hipStream_t);

// out = sigma x on every box node (0 where not an unknown): the caller's buffer.
__global__ void __launch_bounds__(kThreads) k_cg_unscale(L0View<double> v, const double* __restrict__ sigma,
                                                         const double* __restrict__ xv,
                                                         double* __restrict__ out) {
    L0_LOOP_BEGIN
    if (inb) out[n.i] = n.unk ? sigma[n.i] * xv[n.i] : 0.0;
    L0_LOOP_END
}

void cg_unscale(const FineLevel& L, const double* x, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_unscale, l0_grid(L), dim3(kWave, kBlockY), 0, s, L.view<double>(),
                       L.sigma, x, out);
    HIPCHECK(hipGetLastError());
}

__global__ void __launch_bounds__(kMThreads) k_mask_copy(L0View<double> v, const double* __restrict__ a,
                                                        double* __restrict__ b, float* __restrict__ b32) {
    l0_march<double, false, false>(
        v, [&](long) { return 0.0; },
        [&](Idx i, int, int, int, bool, int) { return Vals<double, 1>{{at(a, i)}}; },
        [&](Idx i, Vals<double, 1> f, double, double, int, int, int, bool, int) {
            at(b, i) = f.v[0];
            if (b32) at(b32, i) = (float)f.v[0];
        });
}

void cg_mask_copy(const FineLevel& L, const double* in, double* out, float* out32, hipStream_t s) {
    hipLaunchKernelGGL(k_mask_copy, l0_mgrid(L), dim3(kWave, kMY), 0, s, L.view<double>(), in,
                       out, out32);
    HIPCHECK(hipGetLastError());
}

template <typename T>
__global__ void __launch_bounds__(kMThreads) k_l0_dot(L0View<double> v, const double* __restrict__ a,
                                                     const T* __restrict__ b, double* part) {
    __shared__ double lds[kMThreads / kWave];
    double acc = 0.0;
    l0_march<double, false, false>(
        v, [&](long) { return 0.0; },
        [&](Idx i, int, int, int, bool, int) { return Vals<double, 2>{{at(a, i), (double)at(b, i)}}; },
        [&](long, Vals<double, 2> f, double, double, int, int, int, bool, int) {
            acc += f.v[0] * f.v[1];
        });
    double sb = block_sum(acc, lds);
    if (threadIdx.x == 0 && threadIdx.y == 0) part[blockIdx.x] = sb;
}

template <typename T>
void l0_dot(const FineLevel& L, const double* a, const T* b, double* partials, hipStream_t s) {
    if (L.wide) {
        w_dot<T>(L, a, b, partials, s);
        return;
    }
    hipLaunchKernelGGL((k_l0_dot<T>), l0_mgrid(L), dim3(kWave, kMY), 0, s, L.view<double>(), a,
                       b, partials);
    HIPCHECK(hipGetLastError());
}
template void l0_dot<double>(const FineLevel&, const double*, const double*, double*, hipStream_t);
template void l0_dot<float>(const FineLevel&, const double*, const float*, double*, hipStream_t);

// ================================================================ reporting

__global__ void __launch_bounds__(kThreads) k_l0_export(L0View<double> v, double* out, long nbox) {
    L0_LOOP_BEGIN
    if (inb) {
        double cf[6] = {0, 0, 0, 0, 0, 0};
        double dg = 0.0;
        if (n.unk) {
            dg = 1.0;
            for (int d = 0; d < 6; ++d) cf[d] = n.irr ? v.tcoef(d, n.rank) : v.c[d >> 1];
        }
        out[13 * nbox + n.i] = dg;
        for (int d = 0; d < 6; ++d) out[(long)dir_to_k(d) * nbox + n.i] = cf[d];
    }
    L0_LOOP_END
}

void l0_export_coef(const FineLevel& L, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_l0_export, l0_grid(L), dim3(kWave, kBlockY), 0, s, L.view<double>(), out,
                       L.nbox);
    HIPCHECK(hipGetLastError());
}

}  // namespace saamg
