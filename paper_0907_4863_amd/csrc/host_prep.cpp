// Host-side preparation of a discrete domain (see host_prep.h).
#include "host_prep.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <thread>
#include <vector>

namespace saamg {

// Runs f(lo, hi, t) over [0, n) split into contiguous ranges in order, one per thread (at
// most 16 threads, at least `grain` items each; one range on the calling thread when n is
// small).  f must not throw.
template <class F>
static int host_ranges(long n, long grain, F f) {
    const long hw = std::max(1u, std::thread::hardware_concurrency());
    const int nt = (int)std::max(1L, std::min(std::min(hw, 16L), n / std::max(grain, 1L)));
    if (nt <= 1) {
        f(0L, n, 0);
        return 1;
    }
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t) th.emplace_back([=, &f] { f(n * t / nt, n * (t + 1) / nt, t); });
    for (auto& x : th) x.join();
    return nt;
}

DomainPrep prepare_domain(const saamg_domain* dom, int variant, bool scan_mask) {
    if (!dom || !dom->mask) throw ApiError{SAAMG_INVALID_ARG, "domain or mask is NULL"};
    const int nx = dom->nx, ny = dom->ny, nz = dom->nz;
    if (nx < 3 || ny < 3 || nz < 3) throw ApiError{SAAMG_INVALID_ARG, "box must be at least 3^3"};
    if ((double)nx * ny * nz > 2.0e9) throw ApiError{SAAMG_INVALID_ARG, "box too large"};
    if (!(dom->hx > 0) || !(dom->hy > 0) || !(dom->hz > 0))
        throw ApiError{SAAMG_INVALID_ARG, "grid spacings must be positive"};
    if (variant < SAAMG_VARIANT_CONST || variant > SAAMG_VARIANT_QUAD)
        throw ApiError{SAAMG_INVALID_ARG, "unknown boundary variant"};
    if (dom->n_wall < 0 || (dom->n_wall > 0 && (!dom->wall_node || !dom->wall_dir || !dom->wall_s)))
        throw ApiError{SAAMG_INVALID_ARG, "wall arrays are NULL"};

    DomainPrep D;
    const long nxy = (long)nx * ny, nbox = nxy * nz;
    const uint8_t* m = dom->mask;
    // unknowns: their number, and none on a face of the box
    if (scan_mask) {
        // at least one unknown (the device counts them when it builds the segment masks)
        bool any = false;
        for (long t = 0; t < nbox && !any; ++t) any = m[t] != 0;
        if (!any) throw ApiError{SAAMG_INVALID_ARG, "the domain has no unknowns"};
        // faces: the end planes whole, and of every plane its first and last row and column
        char face[16] = {};
        host_ranges(nz, 64, [&](long k0, long k1, int t) {
            bool f = false;
            for (long k = k0; k < k1 && !f; ++k) {
                const uint8_t* P = m + nxy * k;
                if (k == 0 || k == nz - 1)
                    for (long i = 0; i < nxy && !f; ++i) f = P[i] != 0;
                for (long i = 0; i < nx && !f; ++i) f = P[i] || P[i + (long)nx * (ny - 1)];
                for (long j = 0; j < ny && !f; ++j) f = P[(long)nx * j] || P[(long)nx * j + nx - 1];
            }
            face[t] = f;
        });
        for (char f : face)
            if (f) throw ApiError{SAAMG_INVALID_ARG, "an unknown lies on a face of the box"};
    }

    const bool open = dom->robin_d > 0.0;
    if (dom->robin_d < 0.0 || !std::isfinite(dom->robin_d))
        throw ApiError{SAAMG_INVALID_ARG, "robin_d must be 0 (closed ends) or positive"};
    if (open && scan_mask) {
        if (nz < 4) throw ApiError{SAAMG_INVALID_ARG, "open ends need at least 4 box planes"};
        // end-plane unknowns (planes 1 and nz-2) need an unknown on the inner side
        for (long j = 0; j < ny; ++j)
            for (long i = 0; i < nx; ++i) {
                const long a = i + nx * j + nxy, b = i + nx * j + nxy * (nz - 2);
                if ((m[a] && !m[a + nxy]) || (m[b] && !m[b - nxy]))
                    throw ApiError{SAAMG_INVALID_ARG,
                                   "an open-end unknown has no unknown z-neighbour inside"};
            }
    }

    // wall entries, checked and keyed by (node, direction); the domain builder emits them
    // in that order already, so the sort is usually skipped
    const int64_t nw_in = dom->n_wall;
    const long step[6] = {-1, 1, -(long)nx, (long)nx, -nxy, nxy};
    constexpr long kGrain = 1L << 16;
    HostArr<int64_t> key;
    key.alloc((size_t)nw_in);
    int64_t bad_at[16];
    int bad_kind[16];
    for (int t = 0; t < 16; ++t) bad_at[t] = nw_in;
    host_ranges(nw_in, kGrain, [&](long lo, long hi, int t) {
        for (long e = lo; e < hi; ++e) {
            const int64_t node = dom->wall_node[e];
            const int d = dom->wall_dir[e];
            const double sv = dom->wall_s[e];
            int kind = 0;
            if (node < 0 || node >= nbox || d > 5)
                kind = 1;
            else if (!m[node] || m[node + step[d]])
                kind = 2;
            else if (!(sv > 1e-12) || !(sv <= 1.0))
                kind = 3;
            if (kind) {
                bad_at[t] = e;
                bad_kind[t] = kind;
                return;
            }
            key[e] = node * 8 + d;
        }
    });
    {
        int tb = -1;
        for (int t = 0; t < 16; ++t)
            if (bad_at[t] < nw_in && (tb < 0 || bad_at[t] < bad_at[tb])) tb = t;
        if (tb >= 0) {
            static const char* msg[4] = {
                "", "wall entry out of range",
                "wall entry must name an unknown whose neighbour is not an unknown",
                "wall fraction must lie in (1e-12, 1]"};
            throw ApiError{SAAMG_INVALID_ARG, msg[bad_kind[tb]]};
        }
    }
    char unsorted[16] = {};
    host_ranges(nw_in, kGrain, [&](long lo, long hi, int t) {
        for (long e = std::max(lo, 1L); e < hi && !unsorted[t]; ++e) unsorted[t] = key[e] < key[e - 1];
    });
    const bool sorted = std::none_of(unsorted, unsorted + 16, [](char c) { return c != 0; });
    std::vector<int64_t> order;
    if (!sorted) {
        order.resize(nw_in);
        for (int64_t e = 0; e < nw_in; ++e) order[e] = e;
        std::sort(order.begin(), order.end(), [&](int64_t p, int64_t q) { return key[p] < key[q]; });
    }
    auto at = [&](int64_t r) { return sorted ? r : order[r]; };
    char dup[16] = {};
    host_ranges(nw_in, kGrain, [&](long lo, long hi, int t) {
        for (long r = std::max(lo, 1L); r < hi && !dup[t]; ++r) dup[t] = key[at(r)] == key[at(r - 1)];
    });
    for (char c : dup)
        if (c) throw ApiError{SAAMG_INVALID_ARG, "duplicate wall entry"};

    // near-wall rows in node order: the nodes of cut entries (not for the constant rule)
    // merged with the open-end planes' unknowns.  The entries are cut into ranges that
    // start at a new node; range c owns the nodes from its first entry's node to the next
    // range's, and with them the end-plane unknowns there.  A first pass counts each
    // range's rows, a second writes them at the ranges' offsets.
    std::vector<int64_t> ends;
    if (open)
        for (long k : {1L, (long)nz - 2})
            for (long t = 0; t < nxy; ++t)
                if (m[t + nxy * k]) ends.push_back(t + nxy * k);
    const bool cuts = variant != SAAMG_VARIANT_CONST;
    const long nr = std::max(1L, std::min(16L, (long)(nw_in / kGrain)));
    std::vector<int64_t> rs(nr + 1), nlo(nr + 1);  // entry range starts, owned node ranges
    auto node_of = [&](int64_t r) { return key[at(r)] >> 3; };
    for (long c = 0; c <= nr; ++c) {
        int64_t r = nw_in * c / nr;
        while (r > 0 && r < nw_in && node_of(r) == node_of(r - 1)) ++r;
        rs[c] = (c == 0) ? 0 : std::max(r, rs[c - 1]);
    }
    for (long c = 0; c <= nr; ++c)
        nlo[c] = (c == 0) ? INT64_MIN : (c == nr || rs[c] >= nw_in) ? INT64_MAX : node_of(rs[c]);
    for (long c = 1; c <= nr; ++c) nlo[c] = std::max(nlo[c], nlo[c - 1]);
    // the merge of one range: emit(node) for each row, then frac(dir, s) for its cuts
    auto merge = [&](long c, auto emit, auto frac) {
        size_t ei = std::lower_bound(ends.begin(), ends.end(), nlo[c]) - ends.begin();
        const size_t ee = std::lower_bound(ends.begin(), ends.end(), nlo[c + 1]) - ends.begin();
        int64_t last = -1;
        for (int64_t r = rs[c]; r < rs[c + 1]; ++r) {
            const int64_t e = at(r);
            const double sv = dom->wall_s[e];
            if (!cuts || !(sv < 1.0)) continue;
            const int64_t node = key[e] >> 3;
            while (ei < ee && ends[ei] < node) emit(ends[ei++]);
            if (ei < ee && ends[ei] == node) ++ei;
            if (last != node) {
                emit(node);
                last = node;
            }
            frac((int)(key[e] & 7), sv);
        }
        while (ei < ee) emit(ends[ei++]);
    };
    std::vector<int64_t> cnt(nr + 1, 0);
    host_ranges(nr, 1, [&](long lo, long hi, int) {
        for (long c = lo; c < hi; ++c) {
            int64_t k = 0;
            merge(c, [&](int64_t) { ++k; }, [](int, double) {});
            cnt[c + 1] = k;
        }
    });
    for (long c = 0; c < nr; ++c) cnt[c + 1] += cnt[c];
    D.nw_nodes.alloc((size_t)cnt[nr]);
    D.nw_frac.alloc(6 * (size_t)cnt[nr]);
    host_ranges(nr, 1, [&](long lo, long hi, int) {
        for (long c = lo; c < hi; ++c) {
            int64_t row = cnt[c] - 1;
            merge(
                c,
                [&](int64_t node) {
                    ++row;
                    D.nw_nodes[row] = node;
                    for (int q = 0; q < 6; ++q) D.nw_frac[6 * row + q] = 1.0;
                },
                [&](int d, double sv) { D.nw_frac[6 * row + d] = sv; });
        }
    });
    return D;
}

}  // namespace saamg
