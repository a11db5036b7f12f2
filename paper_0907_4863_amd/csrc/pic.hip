// Particle coupling on either side of the solve (Section 1 and Section 4): cloud-in-cell
// deposition of particle charge to the lattice, and the field E = -grad(phi) interpolated
// back to the particles with the same trilinear weights.
//
// Deposition is deterministic in fp64 without floating-point atomics: particles are
// keyed by lattice cell and stably sorted, and each node sums the particles of its (up
// to) eight adjacent cells in a fixed order.  The gather differences phi centrally at the
// eight corner nodes of each particle's cell.
#include <hipcub/hipcub.hpp>

#include "launch.h"

namespace saamg {

struct PicView {
    int nx, ny, nz, zoff;    // box, and the box plane of the lattice's plane 0
    int nxl, nyl, nzl;       // lattice nodes
    double ox, oy, oz;       // lattice node (0, 0, 0)
    double hx, hy, hz;
    double rob;              // 2 h_z / d for open ends, else 0
};

// Lattice cell of a position and the fractional offsets in it; false if outside.
__device__ inline bool pic_cell(const PicView& v, double px, double py, double pz, int* ci,
                                int* cj, int* ck, double* fx, double* fy, double* fz) {
    const double ux = (px - v.ox) / v.hx, uy = (py - v.oy) / v.hy, uz = (pz - v.oz) / v.hz;
    const double gx = floor(ux), gy = floor(uy), gz = floor(uz);
    // reject before converting, so that far-away particles cannot overflow the cast
    if (!(gx >= 0.0 && gx <= v.nxl - 2 && gy >= 0.0 && gy <= v.nyl - 2 && gz >= 0.0 &&
          gz <= v.nzl - 2))
        return false;
    *ci = (int)gx;
    *cj = (int)gy;
    *ck = (int)gz;
    *fx = ux - gx;
    *fy = uy - gy;
    *fz = uz - gz;
    return true;
}

__global__ void k_pic_keys(PicView v, const double* __restrict__ pos, long n, uint32_t sentinel,
                           uint32_t* __restrict__ key, int32_t* __restrict__ idx) {
    const long p = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (p >= n) return;
    int i, j, k;
    double fx, fy, fz;
    const bool in = pic_cell(v, pos[3 * p], pos[3 * p + 1], pos[3 * p + 2], &i, &j, &k, &fx, &fy, &fz);
    key[p] = in ? (uint32_t)(i + (long)(v.nxl - 1) * (j + (long)(v.nyl - 1) * k)) : sentinel;
    idx[p] = (int32_t)p;
}

__global__ void k_pic_ranges(const uint32_t* __restrict__ key, long n, uint32_t sentinel,
                             int32_t* __restrict__ cstart, int32_t* __restrict__ cend) {
    const long s = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (s >= n) return;
    const uint32_t k = key[s];
    if (k == sentinel) return;
    if (s == 0 || key[s - 1] != k) cstart[k] = (int32_t)s;
    if (s == n - 1 || key[s + 1] != k) cend[k] = (int32_t)(s + 1);
}

// One thread per box node: the charge of the particles in the adjacent cells, weighted.
__global__ void k_pic_deposit(PicView v, const double* __restrict__ pos,
                              const int32_t* __restrict__ idx, const int32_t* __restrict__ cstart,
                              const int32_t* __restrict__ cend, double q, double* __restrict__ rho) {
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const long nbox = (long)v.nx * v.ny * v.nz;
    if (t >= nbox) return;
    const int i = (int)(t % v.nx), j = (int)((t / v.nx) % v.ny), kb = (int)(t / ((long)v.nx * v.ny));
    const int k = kb - v.zoff;  // lattice plane
    double sum = 0.0;
    if (i < v.nxl && j < v.nyl && k >= 0 && k < v.nzl) {
        for (int cz = k - 1; cz <= k; ++cz) {
            if (cz < 0 || cz > v.nzl - 2) continue;
            for (int cy = j - 1; cy <= j; ++cy) {
                if (cy < 0 || cy > v.nyl - 2) continue;
                for (int cx = i - 1; cx <= i; ++cx) {
                    if (cx < 0 || cx > v.nxl - 2) continue;
                    const long c = cx + (long)(v.nxl - 1) * (cy + (long)(v.nyl - 1) * cz);
                    for (int s = cstart[c]; s < cend[c]; ++s) {
                        const long p = idx[s];
                        int a, b, e;
                        double fx, fy, fz;
                        pic_cell(v, pos[3 * p], pos[3 * p + 1], pos[3 * p + 2], &a, &b, &e, &fx, &fy, &fz);
                        const double wx = (i == cx + 1) ? fx : 1.0 - fx;
                        const double wy = (j == cy + 1) ? fy : 1.0 - fy;
                        const double wz = (k == cz + 1) ? fz : 1.0 - fz;
                        sum += q * wx * wy * wz;
                    }
                }
            }
        }
    }
    rho[t] = sum / (v.hx * v.hy * v.hz);
}

// phi at box node (i, j, kb) as the field differences see it: 0 off the domain and beyond
// the box; beyond an open end (the ghost planes) eq. inlet's u(x'') - (2 h_z / d) u(x).
__device__ inline double pic_phi(const PicView& v, const double* __restrict__ phi,
                                 const uint8_t* __restrict__ mask, int i, int j, int kb) {
    if (i < 0 || j < 0 || i >= v.nx || j >= v.ny) return 0.0;
    if (v.rob > 0.0 && (kb == 0 || kb == v.nz - 1)) {
        const int ke = kb == 0 ? 1 : v.nz - 2, ki = kb == 0 ? 2 : v.nz - 3;
        const long e = i + (long)v.nx * (j + (long)v.ny * ke);
        if (!mask[e]) return 0.0;
        const long in = i + (long)v.nx * (j + (long)v.ny * ki);
        return (mask[in] ? phi[in] : 0.0) - v.rob * phi[e];
    }
    if (kb < 0 || kb >= v.nz) return 0.0;
    const long n = i + (long)v.nx * (j + (long)v.ny * kb);
    return mask[n] ? phi[n] : 0.0;
}

__global__ void k_pic_gather(PicView v, const double* __restrict__ phi,
                             const uint8_t* __restrict__ mask, const double* __restrict__ pos,
                             long n, double* __restrict__ E) {
    const long p = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (p >= n) return;
    int ci, cj, ck;
    double fx, fy, fz;
    double ex = 0.0, ey = 0.0, ez = 0.0;
    if (pic_cell(v, pos[3 * p], pos[3 * p + 1], pos[3 * p + 2], &ci, &cj, &ck, &fx, &fy, &fz)) {
        for (int dz = 0; dz < 2; ++dz) {
            const double wz = dz ? fz : 1.0 - fz;
            for (int dy = 0; dy < 2; ++dy) {
                const double wy = dy ? fy : 1.0 - fy;
                for (int dx = 0; dx < 2; ++dx) {
                    const double wx = dx ? fx : 1.0 - fx;
                    const double w = wx * wy * wz;
                    const int i = ci + dx, j = cj + dy, kb = ck + dz + v.zoff;
                    ex += w * (-(pic_phi(v, phi, mask, i + 1, j, kb) - pic_phi(v, phi, mask, i - 1, j, kb)) /
                               (2.0 * v.hx));
                    ey += w * (-(pic_phi(v, phi, mask, i, j + 1, kb) - pic_phi(v, phi, mask, i, j - 1, kb)) /
                               (2.0 * v.hy));
                    ez += w * (-(pic_phi(v, phi, mask, i, j, kb + 1) - pic_phi(v, phi, mask, i, j, kb - 1)) /
                               (2.0 * v.hz));
                }
            }
        }
    }
    E[3 * p] = ex;
    E[3 * p + 1] = ey;
    E[3 * p + 2] = ez;
}

static PicView pic_view(const saamg_pic* P) {
    PicView v;
    v.nx = P->g.nx;
    v.ny = P->g.ny;
    v.nz = P->g.nz;
    v.zoff = P->g.z_offset;
    v.nxl = P->nxl;
    v.nyl = P->nyl;
    v.nzl = P->nzl;
    v.ox = P->g.origin[0];
    v.oy = P->g.origin[1];
    v.oz = P->g.origin[2];
    v.hx = P->g.h[0];
    v.hy = P->g.h[1];
    v.hz = P->g.h[2];
    v.rob = (P->g.robin_d > 0.0 && P->g.z_offset == 1) ? 2.0 * P->g.h[2] / P->g.robin_d : 0.0;
    return v;
}

void pic_deposit(saamg_pic* P, const double* pos, long n, double q, double* rho, hipStream_t s) {
    const PicView v = pic_view(P);
    const uint32_t sentinel = (uint32_t)P->ncell;
    const long nbox = (long)v.nx * v.ny * v.nz;
    if (n > 0) {
        hipLaunchKernelGGL(k_pic_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, v, pos, n,
                           sentinel, P->key, P->idx);
        HIPCHECK(hipGetLastError());
        size_t bytes = P->tmp_bytes;
        HIPCHECK(hipcub::DeviceRadixSort::SortPairs(P->tmp, bytes, P->key, P->key_s, P->idx, P->idx_s,
                                                    (int)n, 0, P->key_bits, s));
    }
    HIPCHECK(hipMemsetAsync(P->cstart, 0, sizeof(int32_t) * P->ncell, s));
    HIPCHECK(hipMemsetAsync(P->cend, 0, sizeof(int32_t) * P->ncell, s));
    if (n > 0) {
        hipLaunchKernelGGL(k_pic_ranges, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, P->key_s,
                           n, sentinel, P->cstart, P->cend);
        HIPCHECK(hipGetLastError());
    }
    hipLaunchKernelGGL(k_pic_deposit, dim3((unsigned)((nbox + 255) / 256)), dim3(256), 0, s, v, pos,
                       P->idx_s, P->cstart, P->cend, q, rho);
    HIPCHECK(hipGetLastError());
}

void pic_gather(saamg_pic* P, const double* phi, const double* pos, long n, double* E, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_pic_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pic_view(P),
                       phi, P->mask, pos, n, E);
    HIPCHECK(hipGetLastError());
}

size_t pic_sort_bytes(long n, int bits) {
    size_t bytes = 0;
    HIPCHECK(hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const uint32_t*)nullptr,
                                                (uint32_t*)nullptr, (const int32_t*)nullptr,
                                                (int32_t*)nullptr, (int)n, 0, bits, (hipStream_t)0));
    return bytes;
}

}  // namespace saamg
