// Host-side launchers of the library's kernels.
#pragma once

#include "common.h"

// Particle-coupling context (grid copy, device mask, sort buffers).
struct saamg_pic {
    int device = 0;
    saamg_grid g{};
    int nxl = 0, nyl = 0, nzl = 0;  // lattice nodes per axis
    long ncell = 0;                 // lattice cells
    int key_bits = 1;
    int64_t cap = 0;                // particle capacity
    uint8_t* mask = nullptr;        // box, nonzero = unknown
    uint32_t *key = nullptr, *key_s = nullptr;
    int32_t *idx = nullptr, *idx_s = nullptr;
    int32_t *cstart = nullptr, *cend = nullptr;
    void* tmp = nullptr;
    size_t tmp_bytes = 0;
};

namespace saamg {

// Scalar slots in the per-solve device array `scal`.
enum Slot {
    S_RHO = 0, S_RHO_PREV, S_ALPHA, S_BETA, S_PQ, S_RR, S_BB, S_R0,
    S_INVN, S_LAM, S_RT, S_LZ_S, S_LZ_SP, S_LZ_B,
    S_XA,  // step length still owed to x (x += S_XA p); 0 after a broken-down step
    S_TOL,   // the solve's tolerance
    S_SKIP,  // nonzero: the queued V-cycle is not needed (the residual passes the test)
    S_AR0 = 18,  // kCgRing slots: the step length of each direction in the ring (fp32 CG)
    S_NSLOTS = S_AR0 + 32
};
// Directions of the CG step kept in a ring (x receives them every kCgRing steps and before
// it is read; see k_cg_xring).  At most 32 directions (cg_ring_len): a solve of up to 32
// steps updates x once (a 22-step solve on a 256 x 256 x 768 box: one pass over x and 22
// fp32 directions instead of two passes, 16 and 6); with 8 a flush took 391 us on that box
// (x and 8 directions, 6.2 TB/s), three per 22-step solve.
constexpr int kCgRing = S_NSLOTS - S_AR0;
// The pending directions of a ring flush: ring slots in the order of their steps.
struct RingSlots {
    int m;
    int slot[kCgRing];
};
// Finalisation ops: how the summed partials update `scal`.
enum FinOp { FIN_STORE = 0, FIN_ALPHA, FIN_RHO_INIT, FIN_RHO, FIN_LZ_ALPHA, FIN_LZ_BETA, FIN_NORM,
             FIN_RESTORE_RHO, FIN_XA_CLEAR, FIN_RR };
// Chebyshev step kinds.  CHEB_NEXT_X (level 0 only) is CHEB_NEXT with the previous
// iterate in place of the previous direction (d = xin - din).
enum ChebMode { CHEB_ZERO1 = 0, CHEB_ZERO2, CHEB_FIRST, CHEB_NEXT, CHEB_NEXT_X };

void pic_deposit(saamg_pic* P, const double* pos, long n, double q, double* rho, hipStream_t s);
void pic_gather(saamg_pic* P, const double* phi, const double* pos, long n, double* E, hipStream_t s);
size_t pic_sort_bytes(long n, int bits);

// Nodes per lane of the level-0 kernels on 16-byte lanes, for values of `bytes` bytes.
constexpr int l0_lanes(int bytes) { return 16 / bytes; }
// fp32 lanes per kernel group: the Chebyshev steps from a zero guess, the later Chebyshev
// steps (which carry the fused r . z partials, so l0_dot_parts follows them, and so does
// the dot of a one-level hierarchy), and the prolongation.  Two nodes per lane measured
// slower for each (256 x 256 x 768 ellipse: zero-guess step 90.7 -> 97.1 us, later steps
// 110.6 / 126.8 -> 114.8 / 132.8 us, prolongation 98.8 -> 111.5 us), unlike the CG step.
constexpr int kChebZeroLanesF = 4;
constexpr int kChebLanesF = 4;
constexpr int kProlongLanesF = 4;
constexpr int cheb_lanes(int bytes, int mode) {
    return bytes == 8 ? 2 : (mode <= CHEB_ZERO2 ? kChebZeroLanesF : kChebLanesF);
}
constexpr int dot_lanes(int bytes) { return bytes == 8 ? 2 : kChebLanesF; }
constexpr int prolong_lanes(int bytes) { return bytes == 8 ? 2 : kProlongLanesF; }
// Number of partial sums (blocks) written by the level-0 reduction kernels of the
// 64-node engine (the Lanczos kernels), and by those on 16-byte lanes with n nodes per lane.
long l0_blocks(const FineLevel& L);
long l0_wblocks(const FineLevel& L, int n);
// Symmetric-part apply of the Lanczos estimate on 16-byte lanes (2 fp64 nodes per lane);
// partials over l0_wblocks(L, 2) blocks.
void w_lz_apply(const FineLevel& L, bool sym, const double* vin, const double* scal, double* u,
                double* partials, hipStream_t s);
// Partial sums (blocks) that the level-0 reduction launchers below write, for the lanes
// each of them runs on (FineLevel::wide: see the launchers): cg_resid, cg_pq (fp32 z or
// not), cg_xr, and the V-cycle's fused r . z (its last Chebyshev step, or l0_dot) in a
// working precision of `bytes` bytes.
long cg_resid_parts(const FineLevel& L);
long cg_pq_parts(const FineLevel& L, bool ring, int bytes);
long cg_xr_parts(const FineLevel& L, bool ring, int bytes);
long l0_dot_parts(const FineLevel& L, int bytes);
int l0_choose_zb(int tx, int nsegx, int ny, int nz);
// 16-byte lanes: whether a box of nx nodes per line uses them by default, and the planes
// per block with n nodes per lane (planes: 0 = automatic, else the option's value, capped)
bool l0_wide_default(int nx);
int l0_wide_zb(const FineLevel& L, int n, int planes);
long lc_blocks(const CoarseLevel& C);

void finalize(const double* partials, long nblk, int nq, double* scal, int op, int dst,
              hipStream_t s);
// scal[S_TOL] = tol, scal[S_SKIP] = 0 (start of a solve)
void scal_start(double* scal, double tol, hipStream_t s);

// Zero `bytes` bytes at p with a kernel on stream s (no memset node, any alignment).
void zero_fill(void* p, size_t bytes, hipStream_t s);

// ---- level 0: build
void l0_scatter_nwidx(int32_t* nwidx, const int64_t* nodes, long n, hipStream_t s);
void l0_build_masks(FineLevel& L, const uint8_t* mask, const int32_t* nwidx, int32_t* cnt_irr,
                    int32_t* cnt_unk, hipStream_t s);
// true when the segment masks unk/irr equal L's
bool l0_same_masks(const FineLevel& L, const uint64_t* unk, const uint64_t* irr, hipStream_t s);
// Exclusive scan of n int32 counts into out (nullable), in int64 (outputs cast to int32);
// total points to scan_words(n) int64 values: the sum goes to total[0], the rest is the
// scan's scratch.
long scan_words(long n);
void exclusive_scan(const int32_t* in, int32_t* out, long n, int64_t* total, hipStream_t s);
// The full table (one row per irregular node, slots from base_full) into tab64 / tab32
// ([2][n_irr][8]) and sigma.
void l0_build_table(FineLevel& L, const uint8_t* mask, const int32_t* nwidx, const double* nwfrac,
                    int variant, double sigma0, double* tab64, float* tab32, hipStream_t s);
// De-duplicated table of L from the full one: sets L.base, L.n_tab, L.tab64, L.tab32
// (reallocated).  Synchronises the stream.
void l0_dedup_table(FineLevel& L, const double* full64, const float* full32, hipStream_t s);
void l0_unknown_list(const FineLevel& L, long* out, hipStream_t s);  // requires n_unknowns slots

// ---- level 0: operators
template <typename T>
void l0_apply(const FineLevel& L, bool trans, const T* x, T* y, hipStream_t s);
void l0_lz_start(const FineLevel& L, double* v, double* partials, hipStream_t s);
void l0_lz_apply(const FineLevel& L, bool sym, const double* v, const double* scal, double* u,
                 double* partials, hipStream_t s);
void l0_lz_update(const FineLevel& L, const double* u, const double* cur, double* prev,
                  const double* scal, double* partials, hipStream_t s);
// fdot: fp64 operand of the fused dot (partials of fdot . xout), used when dot is set
template <typename TF, typename T>
void l0_cheb(const FineLevel& L, int mode, const TF* f, const T* xin, const T* din, T* xout,
             T* dout, double c1, double c2, double c2_0, const double* fdot, double* dot_partials,
             hipStream_t s);
template <typename TF, typename T>
void l0_residual(const FineLevel& L, const TF* f, const T* x, T* r, hipStream_t s);
// fc = P^T r in two passes; y: scratch of at least nx*ny*ceil(nz/3) entries, zero from
// allocation on and used by no other kernel (entries that no unknown reaches are read as 0);
// fd (nullable): D^-1 fc of level 1
template <typename T>
void l0_restrict(const FineLevel& L, const CoarseLevel& C, const T* r, T* y, T* fc, T* fd,
                 double omega, hipStream_t s);
template <typename T>
void l0_prolong(const FineLevel& L, const CoarseLevel& C, const T* v, T* x, double omega,
                hipStream_t s);

// ---- level 0 on 16-byte lanes (wide.hip; FineLevel::wide).  The launchers of fine.hip
// dispatch to these; they take the caller's kernel timer.
template <typename T>
void w_apply(const FineLevel& L, bool trans, const T* x, T* y, hipStream_t s);
template <typename T>
void w_cheb(const FineLevel& L, int mode, const T* f, const T* xin, const T* din, T* xout,
            T* dout, double c1, double c2, double c2_0, const double* fdot, double* dot,
            KTimer& kt);
template <typename T>
void w_residual(const FineLevel& L, const T* f, const T* x, T* r, KTimer& kt);
// returns true when y holds the x-folded sums (one per aggregate x, y, layer)
template <typename T>
bool w_restrict_y(const FineLevel& L, const T* r, T* y, double omega, KTimer& kt);
template <typename T>
void w_prolong(const FineLevel& L, const CoarseLevel& C, const T* vc, T* x, double omega,
               KTimer& kt);
template <typename T>
void w_dot(const FineLevel& L, const double* a, const T* b, double* partials, hipStream_t s);
// Solve start without an initial guess on 16-byte lanes (b 16-byte aligned): b~, x = 0,
// r = b~, its fp32 copy and the partials of cg_resid in one pass.
void w_cg_start(const FineLevel& L, const double* b, double* bs, double* x, double* r,
                double* partials, float* r32, hipStream_t s);
void w_cg_resid(const FineLevel& L, const double* bs, const double* x, double* r, double* partials,
                float* r32, hipStream_t s);
// The CG step on 16-byte lanes (directions in a ring): nodes per lane of its two passes,
// and the arithmetic of the first pass's product in mixed precision.  p . A p only sets
// the step length alpha, and x += alpha p and r -= alpha A p take the same alpha, so its
// rounding leaves r the residual of x; in mixed precision it is formed with the fp32
// level-0 operator (summed in fp64).  r -= alpha A p takes A p in fp64.  Mixed precision
// on the 256 x 256 x 768 ellipse, per step, when the first pass still updated x: 4 nodes
// and an fp64 product 317 + 258 us, 4 nodes fp32 300 + 258, 2 nodes fp64 280 + 225,
// 2 nodes fp32 268 + 225 (the x operands had cost the registers of a wavefront per SIMD).
// Without x the first pass takes 153 us on 2 nodes per lane and 137 us on 4.  fp64 keeps
// 16-byte lanes (2 nodes) and fp64 arithmetic throughout.
using CgDirArith = float;
constexpr int kCgDirLanes = 4;
constexpr int kCgXrLanes = 2;
constexpr int cg_dir_lanes(int bytes) { return bytes == 4 ? kCgDirLanes : 2; }
constexpr int cg_xr_lanes(int bytes) { return bytes == 4 ? kCgXrLanes : 2; }
// Ring length for directions of `bytes` bytes on a box of nbox nodes: kCgRing while the
// ring stays within 8 GiB, down to 2 (x is then updated every other step, which moves
// no more than one update per step).
constexpr long kCgRingBudget = 8L << 30;
inline int cg_ring_len(long nbox, int bytes, int forced = 0) {
    if (forced > 0) return std::min(forced, kCgRing);
    const long k = kCgRingBudget / (std::max(nbox, 1L) * bytes);
    return (int)std::max(2L, std::min<long>(kCgRing, k));
}
// pn = z + beta p (rounded to E) and the partials of pn . A pn; r -= alpha A p with A p
// from the stored direction (r32 nullable); x += alpha_j p_j over a ring's pending
// directions
template <class E>
void w_cg_pdir(const FineLevel& L, const E* z, const E* p, E* pn, const double* scal,
               double* partials, KTimer& kt);
template <class E>
void w_cg_xring(const FineLevel& L, double* x, const E* ring, const double* scal,
                const RingSlots& rs, KTimer& kt);
template <class E>
void w_cg_xr(const FineLevel& L, const E* p, double* r, float* r32, const double* scal,
             double* partials, KTimer& kt);

// ---- level 0: CG (fp64)
void cg_init(const FineLevel& L, const double* b, const double* x0, double* bs, double* x,
             hipStream_t s);
// r32 (nullable): fp32 copy of the residual for the fp32 V-cycle
void cg_resid(const FineLevel& L, const double* bs, const double* x, double* r, double* partials,
              float* r32, hipStream_t s);
// Direction update, the product by A and the partials of p . q in one pass, with the
// q-recursion and an fp64 direction (z in the working precision); cg_xr then takes
// r -= alpha q (one node per lane).  Or (cg_ring: 16-byte lanes) directions in a ring, in
// the working precision, and no q: cg_pdir forms the next direction (p -> pn) with the
// partials of pn . A pn, cg_xr_dir takes r -= alpha A p from the stored direction, and
// cg_xring adds the ring's pending alpha_j p_j to x.
template <typename TZ>
void cg_pq(const FineLevel& L, const TZ* z, double* x, double* p, double* q, const double* scal,
           double* partials, hipStream_t s);
template <class E>
void cg_pdir(const FineLevel& L, const E* z, const E* p, E* pn, const double* scal,
             double* partials, hipStream_t s);
template <class E>
void cg_xring(const FineLevel& L, double* x, const E* ring, const double* scal,
              const RingSlots& rs, hipStream_t s);
bool cg_ring(const FineLevel& L);
void cg_xr(const FineLevel& L, double* r, const double* q, const double* scal, double* partials,
           float* r32, hipStream_t s);
template <class E>
void cg_xr_dir(const FineLevel& L, const E* p, double* r, float* r32, const double* scal,
               double* partials, hipStream_t s);
// x += S_XA p: the update the last step still owes x
template <typename TP>
void cg_xflush(const FineLevel& L, double* x, const TP* p, const double* scal, hipStream_t s);
void cg_unscale(const FineLevel& L, const double* x, double* out, hipStream_t s);
// out = in on the unknowns (out untouched elsewhere)
void cg_mask_copy(const FineLevel& L, const double* in, double* out, float* out32, hipStream_t s);
// partial sums of a . b over level-0 unknowns (one per block of l0_blocks)
template <typename T>
void l0_dot(const FineLevel& L, const double* a, const T* b, double* partials, hipStream_t s);

// ---- levels >= 1
template <typename T>
void lc_apply(const CoarseLevel& C, bool trans, const T* x, T* y, hipStream_t s);
void lc_lz_start(const CoarseLevel& C, double* v, double* partials, hipStream_t s);
void lc_lz_apply(const CoarseLevel& C, const double* v, const double* scal, double* u,
                 double* partials, hipStream_t s);
void lc_lz_update(const CoarseLevel& C, const double* u, const double* cur, double* prev,
                  const double* scal, double* partials, hipStream_t s);
// CHEB_ZERO2 reads D^-1 f from xin
template <typename T>
void lc_cheb(const CoarseLevel& C, int mode, const T* f, const T* xin, const T* din, T* xout,
             T* dout, double c1, double c2, double c2_0, hipStream_t s);
// r = f - A x; rd (nullable) = D^-1 r
template <typename T>
void lc_residual(const CoarseLevel& C, const T* f, const T* x, T* r, T* rd, hipStream_t s);
// out = D^-1 in on every storage node
template <typename T>
void lc_dscale(const CoarseLevel& C, const T* in, T* out, hipStream_t s);
// fc = P^T r from r and rd = D_F^-1 r; r is overwritten; fd (nullable) = D_C^-1 fc
template <typename T>
void lc_restrict(const CoarseLevel& F, const CoarseLevel& C, T* r, const T* rd, T* fc, T* fd,
                 double omega, hipStream_t s);
template <typename T>
void lc_prolong(const CoarseLevel& F, const CoarseLevel& C, const T* v, T* x, double omega,
                hipStream_t s);

// ---- setup of levels >= 1
void rap_from_l0(const FineLevel& L, const CoarseLevel& C, double omega, hipStream_t s);
void rap_from_lc(const CoarseLevel& F, const CoarseLevel& C, double omega, hipStream_t s);
void lc_finish(CoarseLevel& C, int32_t* counts, hipStream_t s);    // invD and unknown count
void lc_to_fp32(CoarseLevel& C, hipStream_t s);
// compressed operator (slots, interior stencil, table) from the full fp64 arrays
void lc_compress(CoarseLevel& C, hipStream_t s);
void l0_to_fp32(FineLevel& L, hipStream_t s);
void lc_unknown_list(const CoarseLevel& C, long* out, int32_t* counter, hipStream_t s);

// ---- coarsest level
void dense_from_l0(const FineLevel& L, const long* cidx, const int32_t* cmap, int nL, double* A,
                   hipStream_t s);
void dense_from_lc(const CoarseLevel& C, const long* cidx, const int32_t* cmap, int nL, double* A,
                   hipStream_t s);
void dense_invert(double* A, int n, hipStream_t s);
void fill_cmap(int32_t* cmap, const long* cidx, int nL, hipStream_t s);
template <typename TF, typename T>
void coarse_solve(const double* Ainv, const long* cidx, int nL, const TF* f, T* x, hipStream_t s);
template <typename TF, typename T>
void coarse_gs(const CoarseLevel& C, const TF* f, T* x, int sweeps, hipStream_t s);
void f2d_copy(const float* a, double* b, long n, hipStream_t s);

// ---- reporting helpers
void l0_export_coef(const FineLevel& L, double* out /* device [27][nbox] */, hipStream_t s);

}  // namespace saamg
