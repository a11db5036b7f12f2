// Level-0 solve kernels on 16-byte lanes.
//
// The same z-march as the 64-node engine of fine.hip, except that every lane holds N
// consecutive nodes of its line (N = 4 in fp32, 2 in fp64) and reads and writes them with
// one 16-byte access, so that a wavefront covers 64 N nodes of a line.  The level-0
// kernels are limited by the rate of vector memory instructions rather than by bytes:
// a fp32 7-point residual on a full 256 x 256 x 768 box, marched as here, measured
// 137.6 us with 4-byte lanes, 121.7 us with 8-byte and 110.0 us with 16-byte lanes
// (5.5 TB/s), with identical results.  This engine issues a quarter (fp32) or half (fp64)
// of the 64-node engine's vector memory instructions per node.  It needs rows that start
// 16-byte aligned (nx a multiple of 4) and lines long enough to fill the lanes; the
// hierarchy decides once (FineLevel::wide).
//
// Tiles: a block of kMY wavefronts takes tx consecutive wavefront spans of a line and
// kMY / tx lines (the 64-node engine's tile mapping, with its XCD-aware block remap), and
// marches zb planes.  The segment words of a wavefront's span (N 64-node segments) for
// planes z0-1 .. z1 are fetched up front, one (plane, segment) pair per lane, which bounds
// the planes per block by 64 / N - 2.
#include "march.h"

namespace saamg {

template <typename E, int N>
struct Vec {
    E v[N];
};

template <typename E, int N>
struct ExtVec {
    typedef E type __attribute__((ext_vector_type(N)));
};

// N consecutive elements at a + k (k.b + k.o a multiple of N): one access.
template <int N, class E>
__device__ __forceinline__ Vec<std::remove_const_t<E>, N> vld(E* a, Idx k) {
    using U = std::remove_const_t<E>;
    using VT = typename ExtVec<U, N>::type;
    const VT t = *reinterpret_cast<const VT*>(&at(a, k));
    Vec<U, N> r;
#pragma unroll
    for (int e = 0; e < N; ++e) r.v[e] = t[e];
    return r;
}
template <int N, class E>
__device__ __forceinline__ Vec<std::remove_const_t<E>, N> vldnt(E* a, Idx k) {
    using U = std::remove_const_t<E>;
    using VT = typename ExtVec<U, N>::type;
    const VT t = __builtin_nontemporal_load(reinterpret_cast<const VT*>(&at(a, k)));
    Vec<U, N> r;
#pragma unroll
    for (int e = 0; e < N; ++e) r.v[e] = t[e];
    return r;
}
template <int N, class E, class V>
__device__ __forceinline__ void vstnt(E* a, Idx k, const V (&v)[N]) {
    using VT = typename ExtVec<E, N>::type;
    VT t;
#pragma unroll
    for (int e = 0; e < N; ++e) t[e] = (E)v[e];
    __builtin_nontemporal_store(t, reinterpret_cast<VT*>(&at(a, k)));
}

template <typename T, int N>
__device__ __forceinline__ Vec<T, N> vzero() {
    Vec<T, N> r;
#pragma unroll
    for (int e = 0; e < N; ++e) r.v[e] = T(0);
    return r;
}

// Where a stencil march reads X.  A source brings a lane's N values with one load per
// array (`ld`, issued a plane ahead and kept in flight as `raw`) and forms the values
// when the plane is stepped (`val`); `ld1` / `val1` do the same for one node.
// XArr: a plain array.
template <class E>
struct XArr {
    using type = E;
    template <int N>
    using raw = Vec<E, N>;
    using raw1 = E;
    const E* a;
    template <int N>
    __device__ __forceinline__ Vec<E, N> ld(Idx k) const { return vld<N>(a, k); }
    __device__ __forceinline__ E ld1(Idx k) const { return at(a, k); }
    template <int N>
    __device__ __forceinline__ Vec<E, N> val(const Vec<E, N>& r) const { return r; }
    __device__ __forceinline__ E val1(E r) const { return r; }
};

// XDir: the next CG direction z + beta p (rounded to E), formed from the preconditioned
// residual z and the previous direction p, both in E (fp32 in mixed precision).  It is
// zero where z and p are.
template <class E>
struct XDir {
    using type = E;
    template <int N>
    struct raw {
        Vec<E, N> z, p;
    };
    struct raw1 {
        E z, p;
    };
    const E* z;
    const E* p;
    double beta;
    __device__ __forceinline__ E dir(E zz, E pp) const {
        return (E)__builtin_fma(beta, (double)pp, (double)zz);
    }
    template <int N>
    __device__ __forceinline__ raw<N> ld(Idx k) const { return raw<N>{vld<N>(z, k), vld<N>(p, k)}; }
    __device__ __forceinline__ raw1 ld1(Idx k) const { return raw1{at(z, k), at(p, k)}; }
    template <int N>
    __device__ __forceinline__ Vec<E, N> val(const raw<N>& r) const {
        Vec<E, N> o;
#pragma unroll
        for (int e = 0; e < N; ++e) o.v[e] = dir(r.z.v[e], r.p.v[e]);
        return o;
    }
    __device__ __forceinline__ E val1(const raw1& r) const { return dir(r.z, r.p); }
};

// Loads of one plane of a wavefront's row (the 16-byte-lane counterpart of PlaneLoads).
template <typename T, class XS, int N, class FV>
struct WPlane {
    unsigned nib;   // unknown bits of the lane's N nodes
    unsigned nibr;  // irregular bits
    int rk0;        // table slot of the lane's first irregular node
    int sp;         // the row's packed span word (wave-uniform; see wmarch)
    int tb0;        // table slot of the row's first irregular node (wave-uniform)
    bool ins1;      // lane inside the row's unknown span (in lanes) in plane z+1
    bool reuse;     // the row's table rows are the previous plane's (staged already)
    long ib;        // box index of the span's first node in this plane (wave-uniform)
    typename XS::template raw<N> nxt, ym, yp;  // X at (z+1), (y-1), (y+1), as loaded
    typename XS::raw1 edge;  // lanes 0 and 63: X beyond the span's ends (0 at the line's ends)
    typename ExtVec<T, 16 / sizeof(T)>::type trow;  // 16 bytes of the row's first table rows
    FV fv;
};

// One 8-value table row (6 used) from 16-byte pieces p[0..].
template <typename T, class TV>
__device__ __forceinline__ void row6(const TV* p, T t[6]) {
    if constexpr (sizeof(T) == 4) {
        const TV a = p[0], b = p[1];
        t[0] = a[0]; t[1] = a[1]; t[2] = a[2]; t[3] = a[3]; t[4] = b[0]; t[5] = b[1];
    } else {
        const TV a = p[0], b = p[1], c = p[2];
        t[0] = a[0]; t[1] = a[1]; t[2] = b[0]; t[3] = b[1]; t[4] = c[0]; t[5] = c[1];
    }
}

// March of a tile on 16-byte lanes.  For every lane with unknowns (FULL: every lane in
// the box of a row with unknowns) the march calls
//   fv = fetch(i, x, y, z, nibr, rk0)          (loads, issued one plane ahead)
//   body(i, fv, c, ax, x, y, z, nib)           (arithmetic and stores)
// where i / x address the lane's first node (fetch: the span-clamped lane's, as in the
// 64-node engine; nibr and rk0 are the lane's own irregular bits and first table slot),
// c holds X at the lane's N nodes and, when STENCIL, ax = (A X) there (TR: A^T X), and
// nib the lane's unknown bits.  Values at nodes that are not unknowns are garbage to be
// masked by the body.  X must be zero at nodes that are not unknowns; it may be null when
// not STENCIL.  end(z, last, x, y) runs on every lane after each plane.
//
// Row bookkeeping is done once per tile: for each plane the lanes holding its N segment
// words reduce them to one packed word (the span of the unknowns in lanes, whether the
// row has unknowns and irregular nodes, and how many irregular nodes), which a plane step
// reads with one broadcast; a lane takes its own segment word with cross-lane permutes.
//
// Table rows (STENCIL, or TAB: the body receives the lane's rows as a last argument): the
// irregular nodes of a row's span have consecutive table slots, so the wavefront reads
// them together, 16 bytes per lane (32 fp32 or 16 fp64 rows per load, the first load
// issued a plane ahead), stages them in its slice of LDS, and each lane reads the rows of
// its own irregular nodes from there.  Reading the rows lane by lane instead issued up to
// 2 N loads per plane and took a quarter of the time of the fp32 stencil kernels.  A row
// whose rows are those of the plane before (its line repeats the line below: the same
// slots) neither loads nor stages them again.
//
// BOTH (with STENCIL and TAB, not TR): an irregular node also applies its row of A^T (same
// slot, staged beside the row of A) to the same neighbour values, without the diagonal,
// and the body receives those sums as an extra argument after ax.
template <typename T, int N, bool STENCIL, bool TR, bool FULL, bool TAB = STENCIL,
          bool BOTH = false, class XS, class Fetch, class Body, class End = NoEnd>
__device__ __forceinline__ void wmarch_x(const L0View<T>& v, const XS xs, Fetch fetch, Body body,
                                         End end = End{}) {
    static_assert(!BOTH || (STENCIL && TAB && !TR), "BOTH applies A and A^T rows");
    static_assert(N == 2 || N == 4, "16-byte lanes of 8- or 4-byte values");
    using TX = typename XS::type;
    using FV = decltype(fetch(Idx{0, 0u}, 0, 0, 0, 0u, 0));
    using WP = WPlane<T, XS, N, FV>;
    using TV = typename ExtVec<T, 16 / sizeof(T)>::type;
    constexpr int W = kWave * N;      // nodes per wavefront span
    constexpr int LPW = kWave / N;    // lanes per 64-bit segment word
    constexpr unsigned NM = (1u << N) - 1u;
    constexpr int RV = (int)sizeof(T) / 2;  // 16-byte pieces per table row
    constexpr int R = kWave / RV;           // table rows per wavefront load
    // packed span word: lo | hi << 8 | any << 16 | irregular << 17 | count << 18
    constexpr int SP_ANY = 1 << 16, SP_IRR = 1 << 17, SP_CNT = 18;
    __shared__ TV tl[kMY][kWave];  // each wavefront's staged table rows
    __shared__ TV tl2[BOTH ? kMY : 1][BOTH ? kWave : 1];  // and of A^T (BOTH)
    if (v.skip && *v.skip != 0.0) return;  // wave-uniform: the whole grid returns
    int ws, y, bz;
    l0_tile(v, &ws, &y, &bz);
    const int lane = threadIdx.x;
    ws = __builtin_amdgcn_readfirstlane(ws);
    y = __builtin_amdgcn_readfirstlane(y);
    const int nws = (v.nx + W - 1) / W;
    if (y < 1 || y > v.ny - 2 || ws >= nws) return;
    const int z0 = max(bz * v.zb, 1), z1 = min(bz * v.zb + v.zb, v.nz - 1);
    if (z0 >= z1) return;
    const long nx = v.nx, nxy = v.nxy;
    const T* tb = TR ? v.tabT : v.tab;
    TV* const stage = tl[threadIdx.y];
    TV* const stage2 = tl2[BOTH ? threadIdx.y : 0];
    // words of (plane k = lane / N, segment j = lane % N) of the span, planes z0-1 .. z1
    uint64_t wu = 0, wr = 0;
    int wb = 0;
    if (lane < (z1 - z0 + 2) * N) {
        const int k = lane / N, j = lane % N;
        const int sgx = ws * N + j;
        if (sgx < v.nsegx) {
            const long sg = ((long)(z0 - 1 + k) * v.ny + y) * v.nsegx + sgx;
            wu = v.unk[sg];
            wr = v.irr[sg];
            wb = v.base[sg];
        }
    }
    if (__ballot(wu != 0) == 0) return;
    const int x0 = ws * W;
    const long rb = x0 + nx * y;  // box index of the span's first node at plane 0
    const long ib_last = rb + nxy * (z1 - 1);
    const int jl = lane / LPW;          // the lane's segment word
    const int sh = (lane % LPW) * N;    // its first bit there
    const int xl = x0 + N * lane;       // x of the lane's first node
    const bool inb = xl < v.nx;
    int spk;  // lane k N: the packed span word of plane k
    {
        const int jj = lane % N;
        int lo = 1 << 20, hi = -1, cnt = (int)__popcll(wr);
        if (wu) {
            lo = jj * 64 + (int)__builtin_ctzll(wu);
            hi = jj * 64 + 63 - (int)__builtin_clzll(wu);
        }
#pragma unroll
        for (int o = 1; o < N; o <<= 1) {
            lo = min(lo, __shfl_xor(lo, o));
            hi = max(hi, __shfl_xor(hi, o));
            cnt += __shfl_xor(cnt, o);
        }
        spk = (hi < 0 ? 0 : ((lo / N) | ((hi / N) << 8) | SP_ANY)) | (cnt ? SP_IRR : 0) |
              (cnt << SP_CNT);
    }
    auto span_word = [&](int k) { return __builtin_amdgcn_readlane(spk, k * N); };
    auto clamp_lane = [&](int sp) { return min(max(lane, sp & 255), (sp >> 8) & 255); };
    auto load_vec = [&](long ibq, int lc) { return xs.template ld<N>(Idx{ibq, (unsigned)(N * lc)}); };
    // 16 bytes of table rows tb0 + c R .. of a row with cnt irregular nodes
    auto load_rows_of = [&](const T* tbx, int tb0, int c, int cnt) {
        TV d;
#pragma unroll
        for (int q = 0; q < 16 / (int)sizeof(T); ++q) d[q] = T(0);
        if (lane < min(cnt - c * R, R) * RV)
            d = *reinterpret_cast<const TV*>(reinterpret_cast<const char*>(tbx + 8 * ((long)tb0 + c * R)) +
                                             (unsigned)lane * 16u);
        return d;
    };
    auto load_rows = [&](int tb0, int c, int cnt) { return load_rows_of(tb, tb0, c, cnt); };
    auto load_plane = [&](int q, long ib) {
        WP P;
        P.ib = ib;
        const int k = q - (z0 - 1);
        P.sp = span_word(k);
        const int lc = clamp_lane(P.sp);
        const int lc1 = clamp_lane(span_word(k + 1));
        P.ins1 = lc1 == lane;
        // the lane's own words, from lane k N + jl
        const int src = (k * N + jl) * 4;
        const uint32_t ulo = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)(uint32_t)wu);
        const uint32_t uhi = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)(uint32_t)(wu >> 32));
        const uint32_t rlo = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)(uint32_t)wr);
        const uint32_t rhi = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)(uint32_t)(wr >> 32));
        const int sb = __builtin_amdgcn_ds_bpermute(src, wb);
        const bool lowh = sh < 32;
        const int shh = lowh ? sh : sh - 32;
        const uint32_t below = (1u << shh) - 1u;
        P.nib = ((lowh ? ulo : uhi) >> shh) & NM;
        P.nibr = ((lowh ? rlo : rhi) >> shh) & NM;
        P.rk0 = sb + (lowh ? (int)__popc(rlo & below) : (int)__popc(rlo) + (int)__popc(rhi & below));
        P.tb0 = __builtin_amdgcn_readlane(wb, k * N);
        const int cnt = P.sp >> SP_CNT;
        P.reuse = q > z0 && cnt <= R && P.tb0 == __builtin_amdgcn_readlane(wb, (k - 1) * N) &&
                  cnt == (span_word(k - 1) >> SP_CNT);
        P.fv = fetch(Idx{ib, (unsigned)(N * lc)}, x0 + N * lc, y, q, P.nibr, P.rk0);
        if (STENCIL) {
            P.nxt = load_vec(ib + nxy, lc1);
            P.ym = load_vec(ib - nx, lc);
            P.yp = load_vec(ib + nx, lc);
            P.edge = typename XS::raw1{};
            if (lane == 0 && x0 > 0) P.edge = xs.ld1(Idx{ib - 1, 0u});
            if (lane == kWave - 1 && x0 + W < v.nx) P.edge = xs.ld1(Idx{ib, (unsigned)W});
        }
        if (TAB) {
#pragma unroll
            for (int e = 0; e < 16 / (int)sizeof(T); ++e) P.trow[e] = T(0);
            if (!P.reuse) P.trow = load_rows(P.tb0, 0, cnt);
        }
        return P;
    };
    Vec<TX, N> zm = vzero<TX, N>(), c = vzero<TX, N>();
    if (STENCIL) {
        int lc = clamp_lane(span_word(0));
        zm = xs.val(load_vec(rb + nxy * (z0 - 1), lc));
        if (lc != lane) zm = vzero<TX, N>();
        lc = clamp_lane(span_word(1));
        c = xs.val(load_vec(rb + nxy * z0, lc));
        if (lc != lane) c = vzero<TX, N>();
    }
    auto settle_plane = [&](const WP& P) {
        if (STENCIL) {
            settle(P.nxt);
            settle(P.ym);
            settle(P.yp);
            settle(P.edge);
        }
        if (TAB) settle(P.trow);
        settle(P.fv);
    };
    auto step = [&](const WP& P, int z) {
        settle_plane(P);
        if (z >= z1) return;
        Vec<TX, N> zp = vzero<TX, N>();
        if (STENCIL && P.ins1) zp = xs.val(P.nxt);
        if (P.sp & SP_ANY) {
            Vec<T, N> cv, ax, tsT;
#pragma unroll
            for (int e = 0; e < N; ++e) {
                cv.v[e] = T(c.v[e]);
                ax.v[e] = T(0);
                tsT.v[e] = T(0);
            }
            // the interior row at every node; irregular nodes are overwritten below
            T left = T(0), right = T(0);
            Vec<TX, N> ymv = vzero<TX, N>(), ypv = vzero<TX, N>();
            if (STENCIL) {
                ymv = xs.val(P.ym);
                ypv = xs.val(P.yp);
                const TX edge = xs.val1(P.edge);
                left = T(wave_shift<true>(c.v[N - 1], edge));
                right = T(wave_shift<false>(c.v[0], edge));
#pragma unroll
                for (int e = 0; e < N; ++e) {
                    const T xm = e ? cv.v[e - 1] : left;
                    const T xp = e < N - 1 ? cv.v[e + 1] : right;
                    ax.v[e] = cv.v[e] + v.c[0] * (xm + xp) + v.c[1] * (T(ymv.v[e]) + T(ypv.v[e])) +
                              v.c[2] * (T(zm.v[e]) + T(zp.v[e]));
                }
            }
            // table rows of the lane's irregular nodes, staged through LDS one wavefront
            // load at a time (one load for rows of up to R irregular nodes).  A stencil
            // kernel applies each row as it reads it, so that one row (6 values) is live
            // at a time instead of N: with N rows held, the fp64 kernels on 4-node lanes
            // needed 137 registers (3 wavefronts per SIMD).
            constexpr int NT = STENCIL ? 1 : N;  // rows handed to the body (TAB && !STENCIL)
            T t[NT][6];
#pragma unroll
            for (int e = 0; e < NT; ++e)
#pragma unroll
                for (int d = 0; d < 6; ++d) t[e][d] = T(0);
            if (TAB && (P.sp & SP_IRR)) {
                const int cnt = P.sp >> SP_CNT;
                for (int ch = 0; ch * R < cnt; ++ch) {
                    if (!P.reuse) {  // (reuse: one load's rows, staged by the plane before)
                        const TV d = ch ? load_rows(P.tb0, ch, cnt) : P.trow;
                        TV dT;
                        if constexpr (BOTH) dT = load_rows_of(v.tabT, P.tb0, ch, cnt);
                        __builtin_amdgcn_wave_barrier();
                        stage[lane] = d;
                        if constexpr (BOTH) stage2[lane] = dT;
                        __builtin_amdgcn_wave_barrier();
                    }
                    int r = P.rk0 - P.tb0 - ch * R;
#pragma unroll
                    for (int e = 0; e < N; ++e) {
                        if ((P.nibr >> e) & 1u) {
                            if (r >= 0 && r < R) {
                                if constexpr (STENCIL) {
                                    T t6[6];
                                    row6<T>(stage + r * RV, t6);
                                    const T xm = e ? cv.v[e - 1] : left;
                                    const T xp = e < N - 1 ? cv.v[e + 1] : right;
                                    ax.v[e] = cv.v[e] + t6[0] * xm + t6[1] * xp + t6[2] * T(ymv.v[e]) +
                                              t6[3] * T(ypv.v[e]) + t6[4] * T(zm.v[e]) +
                                              t6[5] * T(zp.v[e]);
                                    if constexpr (BOTH) {
                                        T u6[6];
                                        row6<T>(stage2 + r * RV, u6);
                                        tsT.v[e] = u6[0] * xm + u6[1] * xp + u6[2] * T(ymv.v[e]) +
                                                   u6[3] * T(ypv.v[e]) + u6[4] * T(zm.v[e]) +
                                                   u6[5] * T(zp.v[e]);
                                    }
                                } else {
                                    row6<T>(stage + r * RV, t[e]);
                                }
                            }
                            ++r;
                        }
                    }
                    __builtin_amdgcn_wave_barrier();
                }
            }
            if (FULL ? inb : P.nib != 0u) {
                if constexpr (TAB && !STENCIL)
                    body(Idx{P.ib, (unsigned)(N * lane)}, P.fv, cv, ax, xl, y, z, P.nib, t);
                else if constexpr (BOTH)
                    body(Idx{P.ib, (unsigned)(N * lane)}, P.fv, cv, ax, tsT, xl, y, z, P.nib);
                else
                    body(Idx{P.ib, (unsigned)(N * lane)}, P.fv, cv, ax, xl, y, z, P.nib);
            }
        }
        if (STENCIL) {
            zm = c;
            c = zp;
        }
        end(z, z == z1 - 1, xl, y);
    };
    long ibz = rb + nxy * z0;
    WP pa = load_plane(z0, ibz);
    for (int z = z0; z < z1; z += 2) {
        const long ib1 = ibz + nxy;
        WP pb = load_plane(min(z + 1, z1 - 1), ib1 < ib_last ? ib1 : ib_last);
        step(pa, z);
        ibz += 2 * nxy;
        pa = load_plane(min(z + 2, z1 - 1), ibz < ib_last ? ibz : ib_last);
        step(pb, z + 1);
    }
}

template <typename T, int N, bool STENCIL, bool TR, bool FULL, bool TAB = STENCIL,
          bool BOTH = false, class TX, class Fetch, class Body, class End = NoEnd>
__device__ __forceinline__ void wmarch(const L0View<T>& v, const TX* __restrict__ X, Fetch fetch,
                                       Body body, End end = End{}) {
    wmarch_x<T, N, STENCIL, TR, FULL, TAB, BOTH>(v, XArr<TX>{X}, fetch, body, end);
}

#define WNOFETCH [&](Idx, int, int, int, unsigned, int) { return NoVals{}; }

template <typename T>
constexpr int kLanes = l0_lanes((int)sizeof(T));

template <typename T>
static inline L0View<T> wview(const FineLevel& L, int n) {
    L0View<T> v = L.view<T>();
    const int nws = (L.nx + kWave * n - 1) / (kWave * n);
    v.tx = nws >= kMY ? kMY : (nws >= 2 ? 2 : 1);
    v.gx = (nws + v.tx - 1) / v.tx;
    v.gy = (L.ny + kMY / v.tx - 1) / (kMY / v.tx);
    v.zb = L.wzb[n == 4 ? 1 : 0];
    return v;
}

static inline long wblocks(const L0View<double>& v, int nz, int zb) {
    return (long)v.gx * v.gy * ((nz + zb - 1) / zb);
}

long l0_wblocks(const FineLevel& L, int n) {
    const L0View<double> v = wview<double>(L, n);
    return wblocks(v, L.nz, v.zb);
}

template <typename T>
static inline dim3 wgrid(const FineLevel& L) {
    return dim3((unsigned)l0_wblocks(L, kLanes<T>));
}

// ---------------------------------------------------------------- operator

// y = A x (TR: A^T x) at the unknowns; other nodes of y untouched (scalar stores in lanes
// that are not all unknowns).
template <typename T, bool TR>
__global__ void __launch_bounds__(kMThreads) k_w_apply(L0View<T> v, const T* __restrict__ xv,
                                                      T* __restrict__ yv) {
    constexpr int N = kLanes<T>;
    wmarch<T, N, true, TR, false>(v, xv, WNOFETCH,
                                  [&](Idx i, NoVals, const Vec<T, N>&, const Vec<T, N>& ax, int,
                                      int, int, unsigned nib) {
                                      if (nib == (1u << N) - 1u) {
                                          vstnt<N>(yv, i, ax.v);
                                      } else {
#pragma unroll
                                          for (int e = 0; e < N; ++e)
                                              if ((nib >> e) & 1u)
                                                  at(yv, Idx{i.b, i.o + (unsigned)e}) = ax.v[e];
                                      }
                                  });
}

template <typename T>
void w_apply(const FineLevel& L, bool trans, const T* x, T* y, hipStream_t s) {
    const L0View<T> v = wview<T>(L, kLanes<T>);
    if (trans)
        hipLaunchKernelGGL((k_w_apply<T, true>), wgrid<T>(L), dim3(kWave, kMY), 0, s, v, x, y);
    else
        hipLaunchKernelGGL((k_w_apply<T, false>), wgrid<T>(L), dim3(kWave, kMY), 0, s, v, x, y);
    HIPCHECK(hipGetLastError());
}
template void w_apply<double>(const FineLevel&, bool, const double*, double*, hipStream_t);
template void w_apply<float>(const FineLevel&, bool, const float*, float*, hipStream_t);

// ---------------------------------------------------------------- Lanczos

// u = S q with q = vin * scal[S_LZ_S] and S the symmetric part (A + A^T)/2, 2 nodes per
// lane (see k_l0_lz_apply); partials of q.u.  Rows whose node is not irregular equal their
// columns, so only irregular nodes (the fetched bits) take the row of A^T too.
template <bool SYM>
__global__ void __launch_bounds__(kMThreads) k_w_lz_apply(L0View<double> v,
                                                         const double* __restrict__ vin,
                                                         const double* __restrict__ scal,
                                                         double* __restrict__ u, double* part) {
    constexpr int N = 2;
    __shared__ double lds[kMThreads / kWave];
    const double sc = scal[S_LZ_S];
    double a0 = 0.0;
    auto irr_bits = [&](Idx, int, int, int, unsigned nibr, int) { return nibr; };
    auto out = [&](Idx i, unsigned nibr, const Vec<double, N>& c, const Vec<double, N>& ax,
                   const Vec<double, N>* ts, unsigned nib) {
        double o[N];
#pragma unroll
        for (int e = 0; e < N; ++e) {
            const double q = sc * c.v[e], aq = sc * ax.v[e];
            double oe = aq;
            if (ts && ((nibr >> e) & 1u)) {
                const double at = q + sc * ts->v[e];
                oe = 0.5 * (aq + at);
            }
            const bool un = (nib >> e) & 1u;
            o[e] = un ? oe : 0.0;
            a0 += un ? q * o[e] : 0.0;
        }
        vstnt<N>(u, i, o);
    };
    if constexpr (SYM)
        wmarch<double, N, true, false, false>(
            v, vin, irr_bits,
            [&](Idx i, unsigned nibr, const Vec<double, N>& c, const Vec<double, N>& ax, int, int,
                int, unsigned nib) { out(i, nibr, c, ax, nullptr, nib); });
    else
        wmarch<double, N, true, false, false, true, true>(
            v, vin, irr_bits,
            [&](Idx i, unsigned nibr, const Vec<double, N>& c, const Vec<double, N>& ax,
                const Vec<double, N>& ts, int, int, int, unsigned nib) {
                out(i, nibr, c, ax, &ts, nib);
            });
    const double s0 = block_sum(a0, lds);
    if (threadIdx.x == 0 && threadIdx.y == 0) part[blockIdx.x] = s0;
}

void w_lz_apply(const FineLevel& L, bool sym, const double* vin, const double* scal, double* u,
                double* partials, hipStream_t s) {
    const L0View<double> v = wview<double>(L, 2);
    const dim3 g((unsigned)l0_wblocks(L, 2));
    if (sym)
        hipLaunchKernelGGL(k_w_lz_apply<true>, g, dim3(kWave, kMY), 0, s, v, vin, scal, u,
                           partials);
    else
        hipLaunchKernelGGL(k_w_lz_apply<false>, g, dim3(kWave, kMY), 0, s, v, vin, scal, u,
                           partials);
    HIPCHECK(hipGetLastError());
}

// ---------------------------------------------------------------- V-cycle

// The Chebyshev steps of fine.hip (same modes and arithmetic), N nodes per lane.
template <typename T, int MODE, bool DOT>
__global__ void __launch_bounds__(kMThreads) k_w_cheb(L0View<T> v, const T* __restrict__ f,
                                                     const T* __restrict__ xin,
                                                     const T* __restrict__ din, T* __restrict__ xout,
                                                     T* __restrict__ dout, T c1, T c2, T c20,
                                                     const double* __restrict__ fdot, double* part) {
    constexpr int N = cheb_lanes((int)sizeof(T), MODE);
    __shared__ double lds[kMThreads / kWave];
    double acc = 0.0;
    constexpr bool LF = MODE == CHEB_FIRST || MODE == CHEB_NEXT || MODE == CHEB_NEXT_X ||
                        MODE == CHEB_ZERO1;
    constexpr bool LD = MODE == CHEB_NEXT || MODE == CHEB_NEXT_X;
    struct R {
        Vec<T, N> f, d;
        Vec<double, N> b;
    };
    auto fetch = [&](Idx i, int, int, int, unsigned, int) {
        R r;
        r.f = LF ? vldnt<N>(f, i) : vzero<T, N>();
        r.d = LD ? vldnt<N>(din, i) : vzero<T, N>();
        r.b = (DOT && fdot) ? vldnt<N>(fdot, i) : vzero<double, N>();
        return r;
    };
    auto body = [&](Idx i, const R& fv, const Vec<T, N>& c, const Vec<T, N>& ax, int, int, int,
                    unsigned nib) {
        T xo[N], dn[N];
#pragma unroll
        for (int e = 0; e < N; ++e) {
            const bool u = (nib >> e) & 1u;
            const T fi = fv.f.v[e];
            T xe, de;
            if (MODE == CHEB_ZERO1) {
                xe = c20 * fi;
                de = xe;
            } else if (MODE == CHEB_ZERO2) {  // c = f, ax = A f
                const T x1 = c20 * c.v[e];
                de = c1 * x1 + c2 * (c.v[e] - c20 * ax.v[e]);
                xe = x1 + de;
            } else {
                const T r = fi - ax.v[e];
                const T dprev = (MODE == CHEB_NEXT_X) ? c.v[e] - fv.d.v[e] : fv.d.v[e];
                de = (MODE == CHEB_FIRST) ? c20 * r : c1 * dprev + c2 * r;
                xe = c.v[e] + de;
            }
            xo[e] = u ? xe : T(0);
            dn[e] = u ? de : T(0);
            if (DOT && u) acc += (fdot ? fv.b.v[e] : (double)fi) * (double)xe;
        }
        vstnt<N>(xout, i, xo);
        if (dout) vstnt<N>(dout, i, dn);
    };
    if (MODE == CHEB_ZERO1)
        wmarch<T, N, false, false, kFullRows<T>>(v, (const T*)nullptr, fetch, body);
    else if (MODE == CHEB_ZERO2)
        wmarch<T, N, true, false, kFullRows<T>>(v, f, fetch, body);
    else
        wmarch<T, N, true, false, kFullRows<T>>(v, xin, fetch, body);
    if (DOT) {
        const double sb = block_sum(acc, lds);
        if (threadIdx.x == 0 && threadIdx.y == 0) part[blockIdx.x] = sb;
    }
}

template <typename T>
void w_cheb(const FineLevel& L, int mode, const T* f, const T* xin, const T* din, T* xout,
            T* dout, double c1, double c2, double c2_0, const double* fdot, double* dot,
            KTimer& kt_) {
    const dim3 b(kWave, kMY);
#define WCHEB_LAUNCH(M)                                                                        \
    {                                                                                          \
        constexpr int n_ = cheb_lanes((int)sizeof(T), M);                                      \
        const L0View<T> v = wview<T>(L, n_);                                                   \
        const dim3 g((unsigned)l0_wblocks(L, n_));                                             \
        if (dot)                                                                               \
            klaunch(kt_, true, (k_w_cheb<T, M, true>), g, b, v, f, xin, din, xout, dout,       \
                    (T)c1, (T)c2, (T)c2_0, fdot, dot);                                         \
        else                                                                                   \
            klaunch(kt_, true, (k_w_cheb<T, M, false>), g, b, v, f, xin, din, xout, dout,      \
                    (T)c1, (T)c2, (T)c2_0, fdot, dot);                                         \
    }
    switch (mode) {
        case CHEB_ZERO1: WCHEB_LAUNCH(CHEB_ZERO1) break;
        case CHEB_ZERO2: WCHEB_LAUNCH(CHEB_ZERO2) break;
        case CHEB_FIRST: WCHEB_LAUNCH(CHEB_FIRST) break;
        case CHEB_NEXT_X: WCHEB_LAUNCH(CHEB_NEXT_X) break;
        default: WCHEB_LAUNCH(CHEB_NEXT) break;
    }
#undef WCHEB_LAUNCH
    HIPCHECK(hipGetLastError());
}
template void w_cheb<double>(const FineLevel&, int, const double*, const double*, const double*,
                             double*, double*, double, double, double, const double*, double*,
                             KTimer&);
template void w_cheb<float>(const FineLevel&, int, const float*, const float*, const float*,
                            float*, float*, double, double, double, const double*, double*,
                            KTimer&);

template <typename T>
__global__ void __launch_bounds__(kMThreads) k_w_residual(L0View<T> v, const T* __restrict__ f,
                                                         const T* __restrict__ xv,
                                                         T* __restrict__ r) {
    constexpr int N = kLanes<T>;
    wmarch<T, N, true, false, kFullRows<T>>(
        v, xv, [&](Idx i, int, int, int, unsigned, int) { return vldnt<N>(f, i); },
        [&](Idx i, const Vec<T, N>& fv, const Vec<T, N>&, const Vec<T, N>& ax, int, int, int,
            unsigned nib) {
            T o[N];
#pragma unroll
            for (int e = 0; e < N; ++e) o[e] = ((nib >> e) & 1u) ? fv.v[e] - ax.v[e] : T(0);
            vstnt<N>(r, i, o);
        });
}

template <typename T>
void w_residual(const FineLevel& L, const T* f, const T* x, T* r, KTimer& kt_) {
    klaunch(kt_, true, (k_w_residual<T>), wgrid<T>(L), dim3(kWave, kMY), wview<T>(L, kLanes<T>),
            f, x, r);
    HIPCHECK(hipGetLastError());
}
template void w_residual<double>(const FineLevel&, const double*, const double*, double*,
                                 KTimer&);
template void w_residual<float>(const FineLevel&, const float*, const float*, float*, KTimer&);

// First pass of the restriction (see k_l0_restrict_y): y = r - w A^T r summed over the
// three planes of each aggregate layer.  FOLD (a line that one wavefront spans): the lanes
// also sum the x-triples of each aggregate, so that one value per (aggregate x, y, layer)
// goes to yz; a lane owns the aggregates whose first node it holds and takes the nodes
// beyond its own from the next lane.  Otherwise one value per (x, y, layer).
template <typename T, bool FOLD>
__global__ void __launch_bounds__(kMThreads) k_w_restrict_y(L0View<T> v, const T* __restrict__ r,
                                                           T* __restrict__ yz, T omega) {
    constexpr int N = kLanes<T>;
    T acc[N];
#pragma unroll
    for (int e = 0; e < N; ++e) acc[e] = T(0);
    const long mxq = (v.nx + 2) / 3;
    wmarch<T, N, true, true, false>(
        v, r, WNOFETCH,
        [&](Idx, NoVals, const Vec<T, N>& c, const Vec<T, N>& atr, int, int, int, unsigned nib) {
#pragma unroll
            for (int e = 0; e < N; ++e)
                if ((nib >> e) & 1u) acc[e] += c.v[e] - omega * atr.v[e];
        },
        [&](int z, bool last, int x, int y) {
            if (z % 3 == 2 || last) {
                if (FOLD) {
                    T nx_[N];  // the next lane's sums (0 past the wavefront)
#pragma unroll
                    for (int e = 0; e < N; ++e) nx_[e] = wave_shift<false>(acc[e], T(0));
                    const long row = mxq * y + mxq * v.ny * (z / 3);
#pragma unroll
                    for (int e = 0; e < N; ++e) {
                        const int xe = x + e;
                        if (xe % 3 == 0 && xe / 3 < mxq) {
                            T s = T(0);
#pragma unroll
                            for (int k = 0; k < 3; ++k) s += (e + k < N) ? acc[e + k] : nx_[e + k - N];
                            yz[row + xe / 3] = s;
                        }
                    }
                } else if (x < v.nx) {
                    vstnt<N>(yz, Idx{(long)v.nx * y + v.nxy * (z / 3), (unsigned)x}, acc);
                }
#pragma unroll
                for (int e = 0; e < N; ++e) acc[e] = T(0);
            }
        });
}

template <typename T>
bool w_restrict_y(const FineLevel& L, const T* r, T* y, double omega, KTimer& kt_) {
    // z-slabs of a multiple of 3 planes, so that no aggregate layer is split between tiles;
    // in fp32 half again as long as the other kernels' (the per-tile preload allows up to
    // 64 / N - 2 planes): on the 256 x 256 x 768 ellipse 12 planes took 80.6 us against 84.1
    // for 6, while fp64 took 133.5 us with 24 planes against 130.1 with 15
    L0View<T> v = wview<T>(L, kLanes<T>);
    const int zr = sizeof(T) == 4 ? 3 * v.zb / 2 : v.zb;
    v.zb = std::max(3, std::min((kWave / kLanes<T> - 2) / 3 * 3, zr / 3 * 3));
    const long blocks = (long)v.gx * v.gy * ((L.nz + v.zb - 1) / v.zb);
    const bool fold = L.nx <= kWave * kLanes<T>;
    if (fold)
        klaunch(kt_, false, (k_w_restrict_y<T, true>), dim3((unsigned)blocks), dim3(kWave, kMY), v,
                r, y, (T)omega);
    else
        klaunch(kt_, false, (k_w_restrict_y<T, false>), dim3((unsigned)blocks), dim3(kWave, kMY), v,
                r, y, (T)omega);
    HIPCHECK(hipGetLastError());
    return fold;
}
template bool w_restrict_y<double>(const FineLevel&, const double*, double*, double, KTimer&);
template bool w_restrict_y<float>(const FineLevel&, const float*, float*, double, KTimer&);

// Prolongation from level 1 (see k_l0_prolong): x += P v = P_tent v - w A (P_tent v).
// A lane's N nodes lie in at most two aggregates along x; with their x-neighbour
// aggregates that is the coarse x-range qx0-1 .. qx0+2 (qx0 = aggregate of the lane's
// first node), read once per aggregate layer together with the y-neighbour values of
// the two own aggregates on a y-face line.  The z-neighbour values are read per face
// plane.  The coarse values are taken at the lane's own nodes (clamped to the box).
template <typename T>
__global__ void __launch_bounds__(kMThreads) k_w_prolong(L0View<T> v, LCView<T> c,
                                                        const T* __restrict__ vc,
                                                        T* __restrict__ xv, T omega) {
    constexpr int N = prolong_lanes((int)sizeof(T));
    struct R {
        T row[4];  // coarse values at x-range qx0-1 .. qx0+2 of the node's layer
        T yn[2];   // y-face lines: the y-neighbour values of aggregates qx0, qx0+1
        T zn[2];   // z-face planes: the z-neighbour values of aggregates qx0, qx0+1
        Vec<T, N> x;
        unsigned irr;  // the lane's irregular bits
    };
    const int lane = threadIdx.x;
    int cqz = -1;
    T crow[4] = {T(0), T(0), T(0), T(0)}, cyn[2] = {T(0), T(0)};
    auto fetch = [&](Idx i, int xc, int y, int z, unsigned nibr, int rk0) {
        // the lane's own first node (xc is the span-clamped lane's), clamped to the box
        const int xs = min(xc - (int)i.o + N * lane, v.nx - N);
        const int qx = xs / 3, qy = y / 3, qz = z / 3;
        const long a = qx + (long)c.sx * (qy + 1) + c.sxy * (qz + 1);  // storage of qx - 1
        const int fy = y - 3 * qy;
        if (qz != cqz) {  // wave-uniform
            cqz = qz;
            // N = 2 reaches qx0+1 at most (nodes qx0 .. qx0+1 have no right face beyond)
#pragma unroll
            for (int j = 0; j < (N == 4 ? 4 : 3); ++j) crow[j] = vc[a + j];
            if (fy != 1) {
                const long o = fy == 0 ? -(long)c.sx : (long)c.sx;
                cyn[0] = vc[a + 1 + o];
                cyn[1] = vc[a + 2 + o];
            }
        }
        R r;
#pragma unroll
        for (int j = 0; j < 4; ++j) r.row[j] = crow[j];
        r.yn[0] = cyn[0];
        r.yn[1] = cyn[1];
        const int zr = z - 3 * qz;
        r.zn[0] = r.zn[1] = T(0);
        if (zr != 1) {
            const long o = zr == 0 ? -c.sxy : c.sxy;
            r.zn[0] = vc[a + 1 + o];
            r.zn[1] = vc[a + 2 + o];
        }
        r.x = vldnt<N>(xv, i);
        r.irr = nibr;
        return r;
    };
    // the table rows come from the march (TAB)
    wmarch<T, N, false, false, kFullRows<T>, true>(
        v, (const T*)nullptr, fetch,
        [&](Idx i, const R& r, const Vec<T, N>&, const Vec<T, N>&, int xl, int y, int z,
            unsigned nib, const T (&t)[N][6]) {
            const int xs = min(xl, v.nx - N);
            const int qx0 = xs / 3, fy = y - 3 * (y / 3), zr = z - 3 * (z / 3);
            T o[N];
#pragma unroll
            for (int e = 0; e < N; ++e) {
                const int x = xs + e, fx = x - 3 * (x / 3);
                // the node's aggregate is row[1] or row[2] (selects, not a runtime index,
                // so that the record stays in registers)
                const bool second = x / 3 != qx0;
                const T c0 = second ? r.row[2] : r.row[1];
                const T cxm = fx == 0 ? (second ? r.row[1] : r.row[0]) : c0;
                const T cxp = fx == 2 ? (second ? r.row[3] : r.row[2]) : c0;
                const T cyf = second ? r.yn[1] : r.yn[0];
                const T czf = second ? r.zn[1] : r.zn[0];
                const T cym = fy == 0 ? cyf : c0;
                const T cyp = fy == 2 ? cyf : c0;
                const T czm = zr == 0 ? czf : c0;
                const T czp = zr == 2 ? czf : c0;
                T apv;
                if ((r.irr >> e) & 1u) {
                    apv = c0 + t[e][0] * cxm + t[e][1] * cxp + t[e][2] * cym + t[e][3] * cyp +
                          t[e][4] * czm + t[e][5] * czp;
                } else {
                    apv = c0 + v.c[0] * (cxm + cxp) + v.c[1] * (cym + cyp) + v.c[2] * (czm + czp);
                }
                o[e] = ((nib >> e) & 1u) ? r.x.v[e] + (c0 - omega * apv) : T(0);
            }
            vstnt<N>(xv, i, o);
        });
}

template <typename T>
void w_prolong(const FineLevel& L, const CoarseLevel& C, const T* vc, T* x, double omega,
               KTimer& kt_) {
    constexpr int n = prolong_lanes((int)sizeof(T));
    klaunch(kt_, true, (k_w_prolong<T>), dim3((unsigned)l0_wblocks(L, n)), dim3(kWave, kMY),
            wview<T>(L, n), C.view<T>(), vc, x, (T)omega);
    HIPCHECK(hipGetLastError());
}
template void w_prolong<double>(const FineLevel&, const CoarseLevel&, const double*, double*,
                                double, KTimer&);
template void w_prolong<float>(const FineLevel&, const CoarseLevel&, const float*, float*, double,
                               KTimer&);

// Partial sums of a . b over the unknowns, on the tiling of the Chebyshev steps that carry
// the fused r . z partials.
template <typename T>
__global__ void __launch_bounds__(kMThreads) k_w_dot(L0View<T> v, const double* __restrict__ a,
                                                    const T* __restrict__ b, double* part) {
    constexpr int N = dot_lanes((int)sizeof(T));
    __shared__ double lds[kMThreads / kWave];
    double acc = 0.0;
    struct R {
        Vec<double, N> a;
        Vec<T, N> b;
    };
    wmarch<T, N, false, false, false>(
        v, (const T*)nullptr,
        [&](Idx i, int, int, int, unsigned, int) { return R{vldnt<N>(a, i), vldnt<N>(b, i)}; },
        [&](Idx, const R& r, const Vec<T, N>&, const Vec<T, N>&, int, int, int, unsigned nib) {
#pragma unroll
            for (int e = 0; e < N; ++e)
                if ((nib >> e) & 1u) acc += r.a.v[e] * (double)r.b.v[e];
        });
    const double sb = block_sum(acc, lds);
    if (threadIdx.x == 0 && threadIdx.y == 0) part[blockIdx.x] = sb;
}

template <typename T>
void w_dot(const FineLevel& L, const double* a, const T* b, double* partials, hipStream_t s) {
    constexpr int n = dot_lanes((int)sizeof(T));
    hipLaunchKernelGGL((k_w_dot<T>), dim3((unsigned)l0_wblocks(L, n)), dim3(kWave, kMY), 0, s,
                       wview<T>(L, n), a, b, partials);
    HIPCHECK(hipGetLastError());
}
template void w_dot<double>(const FineLevel&, const double*, const double*, double*, hipStream_t);
template void w_dot<float>(const FineLevel&, const double*, const float*, double*, hipStream_t);

// ---------------------------------------------------------------- CG (fp64, 2 nodes per lane)

// r = bs - A x; partials of r.r and bs.bs (see k_cg_resid).  ZX: x = 0 (a start without an
// initial guess), so r = bs and the march reads no stencil operand.
template <bool ZX>
__global__ void __launch_bounds__(kMThreads) k_w_cg_resid(L0View<double> v,
                                                         const double* __restrict__ bs,
                                                         const double* __restrict__ xv,
                                                         double* __restrict__ r, double* part,
                                                         float* __restrict__ r32) {
    constexpr int N = 2;
    __shared__ double lds[kMThreads / kWave];
    double a0 = 0.0, a1 = 0.0;
    wmarch<double, N, !ZX, false, false>(
        v, xv, [&](Idx i, int, int, int, unsigned, int) { return vldnt<N>(bs, i); },
        [&](Idx i, const Vec<double, N>& b, const Vec<double, N>&, const Vec<double, N>& ax, int,
            int, int, unsigned nib) {
            double o[N];
#pragma unroll
            for (int e = 0; e < N; ++e) {
                const bool u = (nib >> e) & 1u;
                o[e] = u ? (ZX ? b.v[e] : b.v[e] - ax.v[e]) : 0.0;
                a0 += o[e] * o[e];
                a1 += u ? b.v[e] * b.v[e] : 0.0;
            }
            vstnt<N>(r, i, o);
            if (r32) vstnt<N>(r32, i, o);
        });
    const double s0 = block_sum(a0, lds), s1 = block_sum(a1, lds);
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        part[blockIdx.x] = s0;
        part[gridDim.x + blockIdx.x] = s1;
    }
}

void w_cg_resid(const FineLevel& L, const double* bs, const double* x, double* r, double* partials,
                float* r32, hipStream_t s) {
    if (x)
        hipLaunchKernelGGL(k_w_cg_resid<false>, wgrid<double>(L), dim3(kWave, kMY), 0, s,
                           wview<double>(L, 2), bs, x, r, partials, r32);
    else
        hipLaunchKernelGGL(k_w_cg_resid<true>, wgrid<double>(L), dim3(kWave, kMY), 0, s,
                           wview<double>(L, 2), bs, (const double*)nullptr, r, partials, r32);
    HIPCHECK(hipGetLastError());
}

// Start of a solve without an initial guess, in one pass (2 nodes per lane): b~ = sigma rho b
// as k_cg_init forms it, x = 0, and r = b~ with its fp32 copy and the partials of r.r and
// b~.b~ exactly as k_w_cg_resid<true> forms them (same march, same grid, same order).
__global__ void __launch_bounds__(kMThreads) k_w_cg_start(L0View<double> v,
                                                         const double* __restrict__ sigma,
                                                         const double* __restrict__ b,
                                                         double* __restrict__ bs,
                                                         double* __restrict__ xv,
                                                         double* __restrict__ r, double* part,
                                                         float* __restrict__ r32) {
    constexpr int N = 2;
    __shared__ double lds[kMThreads / kWave];
    double a0 = 0.0, a1 = 0.0;
    struct SB {
        Vec<double, N> sg, b;
    };
    wmarch<double, N, false, false, false>(
        v, (const double*)nullptr,
        [&](Idx i, int, int, int, unsigned, int) { return SB{vldnt<N>(sigma, i), vldnt<N>(b, i)}; },
        [&](Idx i, const SB& f, const Vec<double, N>&, const Vec<double, N>&, int, int, int z,
            unsigned nib) {
            // end-plane rows of open ends are halved, and so is their right-hand side
            const double rho = (z == 1 || z == v.nz - 2) ? v.rho_end : 1.0;
            double o[N], zero[N];
#pragma unroll
            for (int e = 0; e < N; ++e) {
                const bool u = (nib >> e) & 1u;
                const double be = f.sg.v[e] * rho * f.b.v[e];
                o[e] = u ? be : 0.0;
                zero[e] = 0.0;
                a0 += o[e] * o[e];
                a1 += u ? o[e] * o[e] : 0.0;
            }
            vstnt<N>(bs, i, o);
            vstnt<N>(xv, i, zero);
            vstnt<N>(r, i, o);
            if (r32) vstnt<N>(r32, i, o);
        });
    const double s0 = block_sum(a0, lds), s1 = block_sum(a1, lds);
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        part[blockIdx.x] = s0;
        part[gridDim.x + blockIdx.x] = s1;
    }
}

void w_cg_start(const FineLevel& L, const double* b, double* bs, double* x, double* r,
                double* partials, float* r32, hipStream_t s) {
    hipLaunchKernelGGL(k_w_cg_start, wgrid<double>(L), dim3(kWave, kMY), 0, s,
                       wview<double>(L, 2), (const double*)L.sigma, b, bs, x, r, partials, r32);
    HIPCHECK(hipGetLastError());
}

// The CG step on 16-byte lanes, in two passes that share no q = A p vector (N nodes per
// lane and the first pass's arithmetic TA per precision: cg_dir_lanes, CgDirArith).  The
// directions (in E: fp32 in mixed precision, else fp64) live in a ring of buffers.  The
// first pass forms the new direction p_new = z + beta p_old (rounded to E) in the next
// ring buffer, with p_new . A p_new: p_new at the neighbour lines and planes is formed
// from z and p_old as the march reads them (XDir), so A p_new costs no pass of its own;
// neighbouring blocks still read p_old where this block has stored p_new, hence separate
// buffers.  The second recomputes A p in fp64 from the stored direction for
// r -= alpha A p.  x is not touched: it receives alpha_j p_j for the ring's directions in
// one pass (k_cg_xring) when the ring is full and before anything reads it.  Per unknown
// (w = size of E): z w, p_old w read, p_new w written; then p w, r 8 read, r 8 (and r32 4)
// written; and x 16 plus w per direction once per ring.
template <typename TA, int N, class E>
__global__ void __launch_bounds__(kMThreads) k_w_cg_pdir(L0View<TA> v, const E* __restrict__ zv,
                                                        const E* __restrict__ p,
                                                        E* __restrict__ pn,
                                                        const double* __restrict__ scal,
                                                        double* part) {
    __shared__ double lds[kMThreads / kWave];
    const double beta = scal[S_BETA];
    double acc = 0.0;
    wmarch_x<TA, N, true, false, true>(
        v, XDir<E>{zv, p, beta}, WNOFETCH,
        [&](Idx i, NoVals, const Vec<TA, N>& pv, const Vec<TA, N>& ap, int, int, int,
            unsigned nib) {
            E po[N];
#pragma unroll
            for (int e = 0; e < N; ++e) {
                const bool u = (nib >> e) & 1u;
                po[e] = u ? (E)pv.v[e] : E(0);
                acc += u ? (double)pv.v[e] * (double)ap.v[e] : 0.0;
            }
            vstnt<N>(pn, i, po);
        });
    const double sb = block_sum(acc, lds);
    if (threadIdx.x == 0 && threadIdx.y == 0) part[blockIdx.x] = sb;
}

// x += alpha_j p_j over the pending directions j of the ring, in the order of their steps
// (one fused multiply-add per direction and node, as an update per step would take).  A
// plain stream over the box, 4 nodes per thread: the directions and x are zero at the
// nodes that are not unknowns, and so is every alpha_j p_j there.
template <class E>
__global__ void __launch_bounds__(256) k_cg_xring(long n4, double* __restrict__ x,
                                                 const E* __restrict__ ring, long stride,
                                                 const double* __restrict__ scal, RingSlots rs) {
    double a[kCgRing];
#pragma unroll
    for (int j = 0; j < kCgRing; ++j) a[j] = j < rs.m ? scal[S_AR0 + rs.slot[j]] : 0.0;
    using D2 = ExtVec<double, 2>::type;
    using P2 = typename ExtVec<E, 2>::type;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
         i += (long)gridDim.x * blockDim.x) {
        D2* xp = reinterpret_cast<D2*>(x + 4 * i);
        D2 lo = __builtin_nontemporal_load(xp), hi = __builtin_nontemporal_load(xp + 1);
#pragma unroll
        for (int j = 0; j < kCgRing; ++j) {
            if (j < rs.m) {
                const E* pj = ring + rs.slot[j] * stride + 4 * i;
                E q[4];
                if constexpr (sizeof(E) == 4) {
                    using F4 = ExtVec<float, 4>::type;
                    const F4 t = __builtin_nontemporal_load(reinterpret_cast<const F4*>(pj));
                    q[0] = t[0]; q[1] = t[1]; q[2] = t[2]; q[3] = t[3];
                } else {
                    const P2 t0 = __builtin_nontemporal_load(reinterpret_cast<const P2*>(pj));
                    const P2 t1 = __builtin_nontemporal_load(reinterpret_cast<const P2*>(pj) + 1);
                    q[0] = t0[0]; q[1] = t0[1]; q[2] = t1[0]; q[3] = t1[1];
                }
                lo[0] = __builtin_fma(a[j], (double)q[0], lo[0]);
                lo[1] = __builtin_fma(a[j], (double)q[1], lo[1]);
                hi[0] = __builtin_fma(a[j], (double)q[2], hi[0]);
                hi[1] = __builtin_fma(a[j], (double)q[3], hi[1]);
            }
        }
        __builtin_nontemporal_store(lo, xp);
        __builtin_nontemporal_store(hi, xp + 1);
    }
}

// r -= alpha A p (alpha = S_XA; r left as it is when the step broke down), its fp32 copy
// (mixed precision) and partials of r . r.  Whole rows are stored (zero at the nodes that
// are not unknowns).
template <int N, class E>
__global__ void __launch_bounds__(kMThreads) k_w_cg_xr(L0View<double> v, const E* __restrict__ p,
                                                      double* __restrict__ r,
                                                      float* __restrict__ r32,
                                                      const double* __restrict__ scal,
                                                      double* part) {
    __shared__ double lds[kMThreads / kWave];
    const double alpha = scal[S_XA];
    const bool ok = alpha != 0.0;
    double acc = 0.0;
    wmarch<double, N, true, false, true>(
        v, p, [&](Idx i, int, int, int, unsigned, int) { return vldnt<N>(r, i); },
        [&](Idx i, const Vec<double, N>& rv, const Vec<double, N>&, const Vec<double, N>& ap, int,
            int, int, unsigned nib) {
            double ro[N];
            float r3[N];
#pragma unroll
            for (int e = 0; e < N; ++e) {
                const bool u = (nib >> e) & 1u;
                double ri = u ? rv.v[e] : 0.0;
                if (ok) ri = u ? ri - alpha * ap.v[e] : 0.0;
                ro[e] = ri;
                r3[e] = (float)ri;
                acc += ri * ri;
            }
            if (ok) {
                vstnt<N>(r, i, ro);
                if (r32) vstnt<N>(r32, i, r3);
            }
        });
    const double sb = block_sum(acc, lds);
    if (threadIdx.x == 0 && threadIdx.y == 0) part[blockIdx.x] = sb;
}

template <class E>
void w_cg_pdir(const FineLevel& L, const E* z, const E* p, E* pn, const double* scal,
               double* partials, KTimer& kt_) {
    using TA = std::conditional_t<sizeof(E) == 4, CgDirArith, double>;
    constexpr int n = cg_dir_lanes((int)sizeof(E));
    klaunch(kt_, true, (k_w_cg_pdir<TA, n, E>), dim3((unsigned)l0_wblocks(L, n)), dim3(kWave, kMY),
            wview<TA>(L, n), z, p, pn, scal, partials);
    HIPCHECK(hipGetLastError());
}
template void w_cg_pdir<float>(const FineLevel&, const float*, const float*, float*, const double*,
                               double*, KTimer&);
template void w_cg_pdir<double>(const FineLevel&, const double*, const double*, double*,
                                const double*, double*, KTimer&);

template <class E>
void w_cg_xring(const FineLevel& L, double* x, const E* ring, const double* scal,
                const RingSlots& rs, KTimer& kt_) {
    const long n4 = L.nbox / 4;
    const long blocks = std::min<long>((n4 + 255) / 256, 8L * 1024);
    klaunch(kt_, true, k_cg_xring<E>, dim3((unsigned)std::max<long>(blocks, 1)), dim3(256), n4, x,
            ring, L.nbox, scal, rs);
    HIPCHECK(hipGetLastError());
}
template void w_cg_xring<float>(const FineLevel&, double*, const float*, const double*,
                                const RingSlots&, KTimer&);
template void w_cg_xring<double>(const FineLevel&, double*, const double*, const double*,
                                 const RingSlots&, KTimer&);

template <class E>
void w_cg_xr(const FineLevel& L, const E* p, double* r, float* r32, const double* scal,
             double* partials, KTimer& kt_) {
    constexpr int n = cg_xr_lanes((int)sizeof(E));
    klaunch(kt_, true, (k_w_cg_xr<n, E>), dim3((unsigned)l0_wblocks(L, n)), dim3(kWave, kMY),
            wview<double>(L, n), p, r, r32, scal, partials);
    HIPCHECK(hipGetLastError());
}
template void w_cg_xr<float>(const FineLevel&, const float*, double*, float*, const double*,
                             double*, KTimer&);
template void w_cg_xr<double>(const FineLevel&, const double*, double*, float*, const double*,
                              double*, KTimer&);

}  // namespace saamg
