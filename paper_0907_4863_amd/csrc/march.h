// Device helpers shared by the level-0 z-march engines (64-node segments per wavefront,
// and 16-byte lanes): tile mapping, split box indices, streaming loads and stores,
// lane-mask helpers and the load settling the one-plane-ahead pipelines rely on.
#pragma once

#include <type_traits>

#include "launch.h"

namespace saamg {

// Whole-row stores.  A march kernel that stores whole rows writes every in-box lane of a
// row (segment) with unknowns, the extra lanes writing the zero their node already holds,
// so that each store instruction covers whole cache lines instead of being masked to the
// unknowns.  Measured on the 256 x 256 x 768 elliptic pipe: when every level-0 kernel of
// the mixed-precision solve stores whole rows, the CG kernels that read those vectors run
// faster (k_cg_xr -15%, the solve -2%), while in fp64 the wider writes cost the writers
// more than they save (the fp64 V-cycle kernels +1%, k_cg_pq +3%), so fp64 keeps masked
// stores.
template <typename T>
constexpr bool kFullRows = sizeof(T) == 4;

// Segment, line and z-slab of this wavefront: the block's tile (after the XCD-aware
// remap) holds tx consecutive segments of kMY / tx consecutive lines.
template <typename T>
__device__ inline void l0_tile(const L0View<T>& v, int* seg, int* y, int* bz) {
    // block counts fit in 32 bits: unsigned arithmetic keeps the divisions short
    const unsigned b = blockIdx.x, nb = gridDim.x;
    const unsigned q = nb >> 3;
    const unsigned lb = (b < 8 * q) ? (b & 7) * q + (b >> 3) : b;
    const int w = threadIdx.y;
    const unsigned gx = (unsigned)v.gx, gy = (unsigned)v.gy;
    const unsigned t = lb / gx;
    *seg = (int)(lb % gx) * v.tx + w % v.tx;
    *y = (int)(t % gy) * (kMY / v.tx) + w / v.tx;
    *bz = (int)(t / gy);
}

// Box index of a lane's node, split into a wave-uniform part and the lane's offset, so
// that an access through at() addresses memory as a scalar base plus a 32-bit vector
// offset and needs no 64-bit vector address arithmetic.
struct Idx {
    long b;      // wave-uniform
    unsigned o;  // per lane
    __device__ operator long() const { return b + (long)o; }
};
template <class E>
__device__ __forceinline__ E& at(E* a, Idx k) {
    // the byte offset is formed in 32 bits (lane offsets are small)
    using C = std::conditional_t<std::is_const<E>::value, const char, char>;
    return *reinterpret_cast<E*>(reinterpret_cast<C*>(a + k.b) + k.o * (unsigned)sizeof(E));
}

// Store of a solve kernel's output: a nontemporal (streaming) store.  The outputs are
// written once per launch and are far larger than the caches, which then keep the
// stencil rows the march re-reads (measured: the level-0 kernels 1-5% faster).
template <class E, class V>
__device__ __forceinline__ void nts(E* a, Idx k, V v) {
    __builtin_nontemporal_store((E)v, &at(a, k));
}

// Load of an operand a solve kernel reads once per node (not a stencil operand): a
// nontemporal load, for the same reason.  k_cg_pq keeps ordinary loads (slower there).
template <class E>
__device__ __forceinline__ std::remove_const_t<E> ntl(E* a, Idx k) {
    return __builtin_nontemporal_load(&at(a, k));
}

// 64-bit value of lane k of a wavefront, as a wave-uniform (scalar) value.
__device__ inline uint64_t lane_u64(uint64_t v, int k) {
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, k);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), k);
    return ((uint64_t)hi << 32) | lo;
}

// An empty use of every 32-bit word of a loaded record.  The march calls it at the start
// of each plane step so that, on every path through the step (including the ones that
// skip the plane's arithmetic), the plane's loads have landed before the loop goes round.
// Without it a load can still be in flight at the loop back-edge, and the compiler must
// wait for all outstanding loads, the next plane's included, before it reuses that
// load's registers, which serialises the two-plane pipeline.
template <class R>
__device__ __forceinline__ void settle(const R& r) {
    if constexpr (sizeof(R) >= 4) {
        uint32_t w[sizeof(R) / 4];
        __builtin_memcpy(w, &r, sizeof(w));
#pragma unroll
        for (unsigned k = 0; k < sizeof(R) / 4; ++k) asm volatile("" ::"v"(w[k]));
    }
}

// Table row b + o (b wave-uniform, o per lane) of an 8-wide coefficient table: its 6
// values in two 16-byte loads (fp32; the second narrowed to 8 bytes) or three (fp64).
template <typename T>
__device__ __forceinline__ void load_row6(const T* tb, long b, unsigned o, T t[6]) {
    const char* p = reinterpret_cast<const char*>(tb + 8 * b) + (size_t)o * (8 * sizeof(T));
    if constexpr (sizeof(T) == 4) {
        const float4 a = *reinterpret_cast<const float4*>(p);
        const float2 c = *reinterpret_cast<const float2*>(p + 16);
        t[0] = a.x; t[1] = a.y; t[2] = a.z; t[3] = a.w; t[4] = c.x; t[5] = c.y;
    } else {
        const double2 a = *reinterpret_cast<const double2*>(p);
        const double2 c = *reinterpret_cast<const double2*>(p + 16);
        const double2 e = *reinterpret_cast<const double2*>(p + 32);
        t[0] = a.x; t[1] = a.y; t[2] = c.x; t[3] = c.y; t[4] = e.x; t[5] = e.y;
    }
}

// Lane clamped to the span of the set bits of u (u == 0: lane 0).
__device__ inline int span_lane(uint64_t u, int lane) {
    const int lo = u ? (int)__builtin_ctzll(u) : 0;
    const int hi = u ? 63 - (int)__builtin_clzll(u) : 0;
    return min(max(lane, lo), hi);
}

// Whole-wavefront shift by one lane (DPP wave_shr:1 / wave_shl:1): lane l receives
// lane l-1 (UP) or l+1 (down); the lane without a source keeps `edge`.
template <bool UP, class V>
__device__ __forceinline__ V wave_shift(V src, V edge) {
    constexpr int ctrl = UP ? 0x138 : 0x130;
    if constexpr (sizeof(V) == 4) {
        return __builtin_bit_cast(V, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, edge),
                                                                 __builtin_bit_cast(int, src), ctrl,
                                                                 0xf, 0xf, false));
    } else {
        static_assert(sizeof(V) == 8, "4- or 8-byte values");
        const uint64_t s = __builtin_bit_cast(uint64_t, src), e = __builtin_bit_cast(uint64_t, edge);
        const uint32_t lo = __builtin_amdgcn_update_dpp((int)(uint32_t)e, (int)(uint32_t)s, ctrl,
                                                        0xf, 0xf, false);
        const uint32_t hi = __builtin_amdgcn_update_dpp((int)(uint32_t)(e >> 32),
                                                        (int)(uint32_t)(s >> 32), ctrl, 0xf, 0xf,
                                                        false);
        return __builtin_bit_cast(V, ((uint64_t)hi << 32) | lo);
    }
}

// Optional per-plane hook of the march: end(z, last, x, y) after plane z's arithmetic, on
// every lane (x = its node's x, y = the row; last: the tile's final plane).
struct NoEnd {
    __device__ void operator()(int, bool, int, int) const {}
};

// Small fixed-size records for the fetch phase.
template <typename A, int N>
struct Vals {
    A v[N];
};
struct NoVals {};
#define NOFETCH [&](long, int, int, int, bool, int) { return NoVals{}; }

}  // namespace saamg
