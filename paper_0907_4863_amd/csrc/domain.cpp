// Discrete domain of an analytic beam pipe (Section 4, irregular domains): classify the
// lattice nodes of the bounding box and compute, for every unknown next to the wall,
// the fraction s of the spacing at which the wall cuts the grid line (Section 2,
// Figure "boundary").  Each grid line meets these pipes in one open interval, so the
// wall point is the interval end on the side of the outside neighbour.
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "../../include/saamg.h"

namespace {

constexpr double kSnap = 1e-12;    // fractions within kSnap of 1 are taken as 1
constexpr double kOnWall = 1e-12;  // a point inside only by this relative margin is on the wall

struct Pipe {
    int kind;
    double a, b, len, bore_r, cav;

    bool in_bore(double x, double y) const { return x * x + y * y < bore_r * bore_r * (1.0 - kOnWall); }
    bool in_cavity_z(double z) const { return std::fabs(z) < cav * (1.0 - kOnWall); }

    // strict interior test of the continuous pipe (the caps at |z| = len/2 excluded); a
    // point that passes only by rounding lies on the wall and is outside
    bool inside(double x, double y, double z) const {
        const double keep = 1.0 - kOnWall;
        switch (kind) {
            case SAAMG_SHAPE_CYLINDER:
                return x * x + y * y < a * a * keep;
            case SAAMG_SHAPE_ELLIPSE:
                return (x / a) * (x / a) + (y / b) * (y / b) < keep;
            default: {
                const bool cavity =
                    std::fabs(x) < a * keep && std::fabs(y) < b * keep && in_cavity_z(z);
                return cavity || in_bore(x, y);
            }
        }
    }

    // Half-length of the interval the domain occupies on the grid line through (x, y, z)
    // along `axis` (the interval is symmetric about the pipe axis).
    double half_interval(int axis, double x, double y, double z) const {
        if (kind == SAAMG_SHAPE_BOXBORE) {
            if (axis == 2) return in_bore(x, y) ? 0.5 * len : cav;
            if (in_cavity_z(z)) return axis == 0 ? a : b;
            const double o = axis == 0 ? y : x;
            return std::sqrt(std::fmax(bore_r * bore_r - o * o, 0.0));
        }
        if (axis == 2) return 0.5 * len;
        if (kind == SAAMG_SHAPE_CYLINDER) {
            const double o = axis == 0 ? y : x;
            return std::sqrt(std::fmax(a * a - o * o, 0.0));
        }
        if (axis == 0) return a * std::sqrt(std::fmax(1.0 - (y / b) * (y / b), 0.0));
        return b * std::sqrt(std::fmax(1.0 - (x / a) * (x / a), 0.0));
    }
};

inline double coord(double half, int i, int n) {
    return half * (double)(2 * i - (n - 1)) / (double)(n - 1);
}

struct WallEntry {
    int64_t node;
    uint8_t dir;
    double s;
};

// Runs f(lo, hi) over [0, n) split into contiguous ranges, one per thread (at most 16
// threads, at least `grain` items each); the ranges are in order.
template <class F>
void parallel_ranges(int n, int grain, F f) {
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int nt = std::max(1, std::min({(int)std::min(hw, 16u), n / std::max(grain, 1)}));
    if (nt <= 1) {
        f(0, n, 0);
        return;
    }
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t) {
        const int lo = (int)((long)n * t / nt), hi = (int)((long)n * (t + 1) / nt);
        th.emplace_back([=, &f] { f(lo, hi, t); });
    }
    for (auto& x : th) x.join();
}

}  // namespace

extern "C" int saamg_domain_from_shape(int kind, double a, double b, double length, double bore_r,
                                       double cavity_half_len, int nx, int ny, int nz,
                                       int open_ends, uint8_t* mask_out, int64_t wall_cap,
                                       int64_t* wall_node, uint8_t* wall_dir, double* wall_s,
                                       int64_t* n_wall_out, double* h_out) {
    if (kind < SAAMG_SHAPE_CYLINDER || kind > SAAMG_SHAPE_BOXBORE) return SAAMG_INVALID_ARG;
    if (nx < 3 || ny < 3 || nz < 3 || !mask_out || !n_wall_out) return SAAMG_INVALID_ARG;
    if (open_ends != 0 && open_ends != 1) return SAAMG_INVALID_ARG;
    if (!(a > 0) || !(b > 0) || !(length > 0)) return SAAMG_INVALID_ARG;
    if (kind == SAAMG_SHAPE_BOXBORE && (!(bore_r > 0) || !(cavity_half_len > 0)))
        return SAAMG_INVALID_ARG;
    if (wall_cap > 0 && (!wall_node || !wall_dir || !wall_s)) return SAAMG_INVALID_ARG;
    const Pipe p{kind, a, b, length, bore_r, cavity_half_len};
    const long nxy = (long)nx * ny;
    const double h[3] = {2.0 * a / (nx - 1), 2.0 * b / (ny - 1), length / (nz - 1)};
    if (h_out) {
        for (int q = 0; q < 3; ++q) h_out[q] = h[q];
        h_out[3] = open_ends ? 0.5 * length : 0.0;  // eq. inlet: d = half the pipe length
    }
    // box planes: the lattice's plane k sits at box plane k + open_ends; with open ends the
    // lattice's end planes hold unknowns and the box gains one ghost plane at each end
    const int nzb = nz + 2 * open_ends;
    auto lattice_plane = [&](int kb) { return kb - open_ends; };
    auto unknown_plane = [&](int k) { return open_ends ? (k >= 0 && k < nz) : (k > 0 && k < nz - 1); };

    // The box planes are split into contiguous ranges over threads: first the mask, then
    // (after every plane's mask is known) the wall entries of each range in node order,
    // concatenated in range order.
    parallel_ranges(nzb, 4, [&](int kb0, int kb1, int) {
        for (int kb = kb0; kb < kb1; ++kb) {
            const int k = lattice_plane(kb);
            const double z = coord(0.5 * length, k, nz);
            for (int j = 0; j < ny; ++j) {
                const double y = coord(b, j, ny);
                for (int i = 0; i < nx; ++i) {
                    const double x = coord(a, i, nx);
                    const bool interior_index =
                        i > 0 && j > 0 && i < nx - 1 && j < ny - 1 && unknown_plane(k);
                    mask_out[i + nx * (long)j + nxy * kb] =
                        (interior_index && p.inside(x, y, z)) ? 1 : 0;
                }
            }
        }
    });

    const long step[3] = {1, (long)nx, nxy};
    std::vector<std::vector<WallEntry>> parts(16);
    std::vector<int> bad(16, 0);
    const int nin = std::max(nzb - 2, 0);  // planes 1 .. nzb-2
    parallel_ranges(nin, 4, [&](int r0, int r1, int t) {
        std::vector<WallEntry>& out = parts[t];
        for (int kb = 1 + r0; kb < 1 + r1; ++kb) {
            const int k = lattice_plane(kb);
            const double z = coord(0.5 * length, k, nz);
            for (int j = 1; j < ny - 1; ++j) {
                const double y = coord(b, j, ny);
                for (int i = 1; i < nx - 1; ++i) {
                    const long idx = i + nx * (long)j + nxy * kb;
                    if (!mask_out[idx]) continue;
                    const double x = coord(a, i, nx);
                    const double pos[3] = {x, y, z};
                    for (int d = 0; d < 6; ++d) {
                        const int axis = d / 2;
                        const long nb = (d & 1) ? idx + step[axis] : idx - step[axis];
                        if (mask_out[nb]) continue;
                        // the ghost planes beyond open ends are not walls
                        if (open_ends && axis == 2 && (kb + ((d & 1) ? 1 : -1) == 0 ||
                                                       kb + ((d & 1) ? 1 : -1) == nzb - 1))
                            continue;
                        const double end = p.half_interval(axis, x, y, z);
                        const double wall = (d & 1) ? end : -end;
                        double sv = std::fabs(wall - pos[axis]) / h[axis];
                        if (sv > 1.0 - kSnap) sv = 1.0;
                        if (!(sv > 0.0)) {
                            bad[t] = 1;
                            return;
                        }
                        if (sv < 1.0) out.push_back({idx, (uint8_t)d, sv});
                    }
                }
            }
        }
    });
    for (int t = 0; t < 16; ++t)
        if (bad[t]) return SAAMG_INVALID_ARG;
    int64_t count = 0;
    for (const auto& part : parts) {
        for (const WallEntry& e : part) {
            if (count < wall_cap) {
                wall_node[count] = e.node;
                wall_dir[count] = e.dir;
                wall_s[count] = e.s;
            }
            ++count;
        }
    }
    *n_wall_out = count;
    return count > wall_cap && wall_cap > 0 ? SAAMG_INVALID_ARG : SAAMG_OK;
}
