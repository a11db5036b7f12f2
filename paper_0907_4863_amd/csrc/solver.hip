// Host driver: hierarchy setup and numeric re-setup, V-cycle, PCG state machine and the
// C interface.
//
// Paper: Section 2 (operator and scaling), Section 3 (PCG with an SA-AMG V-cycle,
// Algorithm 1), Table 1 (coarse size limit 1000), Section 5 (relative-residual stop),
// Section 5.2 (reuse of the aggregation hierarchy, Gauss-Seidel coarse level solver).
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "launch.h"

namespace saamg {

static thread_local std::string g_err;
thread_local const double* g_vskip = nullptr;

void hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) throw HipError{e, what};
}

// Device memory of the running entry point: the hierarchy's allocator (the options'
// callbacks, else hipMalloc / hipFree) and the stream its work is queued on.  Set for the
// duration of each entry point by MemScope.
static thread_local MemCtx g_mem{};

MemScope::MemScope(const MemCtx& m, hipStream_t s) : saved(g_mem) {
    g_mem = m;
    g_mem.s = s;
}
MemScope::~MemScope() { g_mem = saved; }

__global__ void k_zero_fill(char* __restrict__ p, size_t bytes) {
    const size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    // bytes before the first 16-byte boundary, the 16-byte body, and the tail
    const size_t head = (16 - ((uintptr_t)p & 15)) & 15;
    const size_t h = head < bytes ? head : bytes;
    const size_t n16 = (bytes - h) / 16;
    if (t < n16) ((uint4*)(p + h))[t] = make_uint4(0u, 0u, 0u, 0u);
    if (t < h) p[t] = 0;
    const size_t tail0 = h + 16 * n16;
    if (t < bytes - tail0) p[tail0 + t] = 0;
}

void zero_fill(void* p, size_t bytes, hipStream_t s) {
    if (!p || bytes == 0) return;
    const size_t threads = std::max<size_t>((bytes + 15) / 16, 16);
    hipLaunchKernelGGL(k_zero_fill, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s,
                       (char*)p, bytes);
    HIPCHECK(hipGetLastError());
}

// The library's own device memory (no allocator callback): a pool per device.  A freed
// block keeps an event recorded on the freeing stream after everything queued there, and
// is handed out again (for a request of the same size class) only once that event has
// completed, so a block is never reused while queued work may still touch it, whatever
// stream the next user runs on.  New memory comes from hipMalloc; nothing is given back
// to the device until the cached bytes exceed kPoolCap, so steady-state setups and solve
// states make no hipMalloc and no device-synchronising hipFree.
namespace {
constexpr size_t kPoolCap = size_t(16) << 30;

struct PoolBlock {
    void* p;
    hipEvent_t ev;
};

struct DevicePool {
    std::multimap<size_t, PoolBlock> free_;     // by size class
    std::unordered_map<void*, size_t> live_;    // block -> size class
    std::vector<hipEvent_t> events_;            // spare events
    size_t cached = 0;
};

std::mutex g_pool_mu;
std::map<int, DevicePool> g_pools;

// Size classes: multiples of 256 B below 64 KiB, above that the next of 2^k * {1, 5/4,
// 3/2, 7/4} (at most 25% slack).
size_t size_class(size_t b) {
    if (b <= (size_t(64) << 10)) return (b + 255) & ~size_t(255);
    size_t k = size_t(1) << (63 - __builtin_clzll(b));
    for (size_t q : {k, k + k / 4, k + k / 2, k + 3 * k / 4, 2 * k})
        if (q >= b) return q;
    return 2 * k;
}

void* pool_alloc(size_t bytes) {
    int dev = 0;
    HIPCHECK(hipGetDevice(&dev));
    const size_t cls = size_class(bytes);
    {
        std::lock_guard<std::mutex> g(g_pool_mu);
        DevicePool& P = g_pools[dev];
        auto range = P.free_.equal_range(cls);
        for (auto it = range.first; it != range.second; ++it) {
            const hipError_t q = hipEventQuery(it->second.ev);
            if (q == hipErrorNotReady) continue;
            (void)hipGetLastError();
            void* p = it->second.p;
            P.events_.push_back(it->second.ev);
            P.free_.erase(it);
            P.cached -= cls;
            P.live_[p] = cls;
            return p;
        }
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, cls);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw ApiError{SAAMG_NOMEM, "hipMalloc of " + std::to_string(cls) + " bytes failed"};
    }
    std::lock_guard<std::mutex> g(g_pool_mu);
    g_pools[dev].live_[p] = cls;
    return p;
}

void pool_free(void* p, hipStream_t s) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::vector<void*> give_back;
    {
        std::lock_guard<std::mutex> g(g_pool_mu);
        DevicePool& P = g_pools[dev];
        auto it = P.live_.find(p);
        if (it == P.live_.end()) {
            (void)hipFree(p);  // not a pool block
            return;
        }
        const size_t cls = it->second;
        P.live_.erase(it);
        hipEvent_t ev = nullptr;
        if (!P.events_.empty()) {
            ev = P.events_.back();
            P.events_.pop_back();
        } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            ev = nullptr;
        }
        if (!ev || hipEventRecord(ev, s) != hipSuccess) {
            (void)hipGetLastError();
            if (ev) P.events_.push_back(ev);
            give_back.push_back(p);  // hipFree waits for the device itself
        } else {
            P.free_.insert({cls, PoolBlock{p, ev}});
            P.cached += cls;
            // over the cap: give back the largest cached blocks
            while (P.cached > kPoolCap && !P.free_.empty()) {
                auto last = std::prev(P.free_.end());
                give_back.push_back(last->second.p);
                P.events_.push_back(last->second.ev);
                P.cached -= last->first;
                P.free_.erase(last);
            }
        }
    }
    for (void* q : give_back) (void)hipFree(q);
}
}  // namespace

// New buffers are zero-filled on the entry point's stream, in stream order with the work
// that follows (a null-stream fill would not be ordered with a non-blocking stream).  The
// fill is a kernel, not a memset, so that no memset node enters a captured graph.
void* dmalloc(size_t bytes) {
    void* p = nullptr;
    if (bytes == 0) bytes = 8;
    if (g_mem.alloc) {
        p = g_mem.alloc(g_mem.ctx, bytes, (void*)g_mem.s);
        if (!p)
            throw ApiError{SAAMG_NOMEM, "the allocator returned NULL for " + std::to_string(bytes) +
                                            " bytes"};
        // the level-0 kernels read and write 16 bytes per lane
        if (reinterpret_cast<uintptr_t>(p) & 255u) {
            g_mem.free(g_mem.ctx, p, (void*)g_mem.s);
            throw ApiError{SAAMG_INVALID_ARG, "the allocator returned memory not aligned to 256 bytes"};
        }
    } else {
        p = pool_alloc(bytes);
    }
    if (g_mem.fill) {
        try {
            zero_fill(p, bytes, g_mem.s);
        } catch (...) {
            dfree(p);
            throw;
        }
    }
    return p;
}

// The caller guarantees that no queued work still uses p (the library synchronises the
// stream before it frees a temporary).
void dfree(void* p) {
    if (!p) return;
    if (g_mem.free)
        g_mem.free(g_mem.ctx, p, (void*)g_mem.s);
    else
        pool_free(p, g_mem.s);
}

ChebCoef cheb_coefficients(double lam_hi, double ratio, int degree) {
    ChebCoef c{};
    c.degree = degree;
    const double lo = lam_hi / ratio;
    const double theta = 0.5 * (lam_hi + lo), delta = 0.5 * (lam_hi - lo);
    const double s1 = theta / delta;
    double rho = 1.0 / s1;
    c.c1[0] = 0.0;
    c.c2[0] = 1.0 / theta;
    for (int k = 1; k < degree; ++k) {
        const double rn = 1.0 / (2.0 * s1 - rho);
        c.c1[k] = rn * rho;
        c.c2[k] = 2.0 * rn / delta;
        rho = rn;
    }
    return c;
}

static double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// ------------------------------------------------------------------ V-cycle buffers

template <typename T>
struct VBuf {
    std::vector<T*> f, xa, xb, d;  // per level; level 0 has no f (the PCG residual is read)
    T* yz = nullptr;               // level-0 restriction scratch (aggregate-plane sums)
    static long yz_size(const saamg_hierarchy* H) {
        return H->l0.nxy * ((H->l0.nz + 2) / 3);
    }
    void alloc(const saamg_hierarchy* H) {
        const int L = H->n_levels;
        f.assign(L, nullptr);
        xa.assign(L, nullptr);
        xb.assign(L, nullptr);
        d.assign(L, nullptr);
        for (int l = 0; l < L; ++l) {
            const long n = (l == 0) ? H->l0.nbox : H->lc[l - 1].nstore;
            xa[l] = (T*)dmalloc(sizeof(T) * n);
            if (l < L - 1) {
                xb[l] = (T*)dmalloc(sizeof(T) * n);
                d[l] = (T*)dmalloc(sizeof(T) * n);
            }
            if (l > 0) f[l] = (T*)dmalloc(sizeof(T) * n);
        }
        if (L > 1) yz = (T*)dmalloc(sizeof(T) * yz_size(H));
    }
    void release() {
        for (auto* v : {&f, &xa, &xb, &d})
            for (T* p : *v) dfree(p);
        dfree(yz);
        yz = nullptr;
        f.clear();
        xa.clear();
        xb.clear();
        d.clear();
    }
    int64_t bytes(const saamg_hierarchy* H) const {
        int64_t b = 0;
        for (int l = 0; l < H->n_levels; ++l) {
            const long n = (l == 0) ? H->l0.nbox : H->lc[l - 1].nstore;
            int cnt = 1 + (l < H->n_levels - 1 ? 2 : 0) + (l > 0 ? 1 : 0);
            b += (int64_t)cnt * n * sizeof(T);
        }
        if (H->n_levels > 1) b += (int64_t)yz_size(H) * sizeof(T);
        return b;
    }
};

template <typename T>
static void chebstep(const saamg_hierarchy* H, int l, int mode, const T* f0, const T* fl,
                     const T* xin, const T* din, T* xout, T* dout, double c1, double c2, double c20,
                     const double* fdot, double* dot, hipStream_t s) {
    if (l == 0)
        l0_cheb<T, T>(H->l0, mode, f0, xin, din, xout, dout, c1, c2, c20, fdot, dot, s);
    else
        lc_cheb<T>(H->lc[l - 1], mode, fl, xin, din, xout, dout, c1, c2, c20, s);
}

// Algorithm 1 on level l with a zero initial guess; returns the buffer holding x_l.  On
// level 0 the right-hand side is the PCG residual f0 in the working precision and the
// result goes to `out`, with partial sums of fdot . out in `dot` (nullable; fdot is the
// fp64 residual).
template <typename T>
static T* vcycle(const saamg_hierarchy* H, VBuf<T>& B, int l, const T* f0, T* out,
                 const double* fdot, double* dot, hipStream_t s) {
    const bool fine = (l == 0);
    // Levels below 1 are latency-bound: their kernels do not wait on the skip flag (a
    // dependent load at each kernel start costs more there than the skipped work).
    VSkipScope vs(l >= 2 ? nullptr : g_vskip);
    if (l == H->n_levels - 1) {
        T* x = fine ? out : B.xa[l];
        if (fine) {
            coarse_solve<T, T>(H->Ainv, H->cidx, H->nL, f0, x, s);
            if (dot) l0_dot<T>(H->l0, fdot, x, dot, s);
        } else if (H->opt.coarse_solver == SAAMG_COARSE_GS) {
            coarse_gs<T, T>(H->lc[l - 1], B.f[l], x, H->opt.coarse_sweeps, s);
        } else {
            coarse_solve<T, T>(H->Ainv, H->cidx, H->nL, B.f[l], x, s);
        }
        return x;
    }
    const LevelParams& P = H->par[l];
    const ChebCoef& c = P.cheb;
    const T* fl = fine ? nullptr : B.f[l];
    T* x = B.xa[l];
    T* other = B.xb[l];
    T* d = B.d[l];
    // pre-smoothing from a zero guess
    if (c.degree == 1) {
        chebstep<T>(H, l, CHEB_ZERO1, f0, fl, nullptr, nullptr, x, nullptr, 0, 0, c.c2[0],
                    nullptr, nullptr, s);
    } else {
        // on levels >= 1 the restriction left D^-1 f in `other`
        chebstep<T>(H, l, CHEB_ZERO2, f0, fl, fine ? nullptr : other, nullptr, x,
                    c.degree > 2 ? d : nullptr, c.c1[1], c.c2[1], c.c2[0], nullptr, nullptr, s);
        for (int k = 2; k < c.degree; ++k) {
            chebstep<T>(H, l, CHEB_NEXT, f0, fl, x, d, other, d, c.c1[k], c.c2[k], c.c2[0],
                        nullptr, nullptr, s);
            std::swap(x, other);
        }
    }
    // residual and restriction; D^-1 f of level l+1 goes to its `other` buffer (the
    // coarsest level has none and needs none)
    T* fd = (l + 1 < H->n_levels - 1) ? B.xb[l + 1] : nullptr;
    if (fine) {
        l0_residual<T, T>(H->l0, f0, x, other, s);
        l0_restrict<T>(H->l0, H->lc[0], other, B.yz, B.f[1], fd, P.omega, s);
    } else {
        lc_residual<T>(H->lc[l - 1], fl, x, other, d, s);
        lc_restrict<T>(H->lc[l - 1], H->lc[l], other, d, B.f[l + 1], fd, P.omega, s);
    }
    T* v = vcycle<T>(H, B, l + 1, nullptr, nullptr, nullptr, nullptr, s);
    // coarse-grid correction
    if (fine)
        l0_prolong<T>(H->l0, H->lc[0], v, x, P.omega, s);
    else
        lc_prolong<T>(H->lc[l - 1], H->lc[l], v, x, P.omega, s);
    // post-smoothing.  Degree 2 on level 0: the second step takes its previous direction as
    // the difference of the two iterates (both still held), so the first stores none.
    const bool xdiff = fine && c.degree == 2;
    for (int k = 0; k < c.degree; ++k) {
        const bool last = (k == c.degree - 1);
        T* dst = (last && fine) ? out : other;
        if (xdiff && k == 1)
            chebstep<T>(H, l, CHEB_NEXT_X, f0, fl, x, other, dst, nullptr, c.c1[k], c.c2[k],
                        c.c2[0], fdot, dot, s);
        else
            chebstep<T>(H, l, k == 0 ? CHEB_FIRST : CHEB_NEXT, f0, fl, x, d, dst,
                        (last || xdiff) ? nullptr : d, c.c1[k], c.c2[k], c.c2[0], fdot,
                        (last && fine) ? dot : nullptr, s);
        other = x;
        x = dst;
    }
    return x;
}

}  // namespace saamg

using namespace saamg;

// ------------------------------------------------------------------ solve state

struct saamg_state {
    saamg_hierarchy* H = nullptr;
    hipStream_t s = nullptr;
    double tol = 1e-8;
    int max_iter = 0;
    bool mixed = false;
    double *x = nullptr, *r = nullptr, *q = nullptr, *bs = nullptr;
    float* r32 = nullptr;  // fp32 copy of r (mixed precision)
    void* z = nullptr;     // preconditioned residual (fp32 in mixed precision)
    void* p = nullptr;     // direction of the fused form (fp64)
    // ring form (cg_ring): the last `ringk` directions in the working precision (`pw`
    // bytes), ring slot k % ringk holding step k's; x has received alpha_j p_j for all but
    // the last `pend` of them.  q is then only the scratch of a final true residual.
    void* ring = nullptr;
    int ringk = 0, pend = 0, pw = 8;
    long kdir = 0;  // directions formed so far in this solve
    bool ringf = false;
    VBuf<float> vf;
    VBuf<double> vd;
    double* part = nullptr;
    long npart = 0;
    double* scal = nullptr;
    double* hscal = nullptr;  // pinned, or hbuf for a state that allocates nothing on the host
    double hbuf[S_NSLOTS] = {};
    hipEvent_t ev = nullptr;  // null: the host waits on the stream instead
    int iter = 0, status = SAAMG_OK, done = 0, repl = 0;
    bool inflight = false;  // a step is queued whose scalars the host has not read yet
    double bnorm = 0, rel_true = 0, rel_rec = 0;
    double t_ms = 0;
    std::chrono::steady_clock::time_point t0;
    int64_t bytes = 0;
};

namespace saamg {

// The level-0 operator of the CG iteration: the hierarchy's own, or the one a later
// saamg_set_operator gave it (the preconditioner then keeps the hierarchy's).
static const FineLevel& cg_op(const saamg_hierarchy* H) { return H->op ? *H->op : H->l0; }

// Ring slot of direction k (k = -1: the one the first step reads) of a ring-form state.
static int ring_index(const saamg_state* S, long k) {
    return (int)(((k % S->ringk) + S->ringk) % S->ringk);
}
template <class E>
static E* ring_at(const saamg_state* S, long k) {
    return (E*)S->ring + (long)ring_index(S, k) * S->H->l0.nbox;
}

// x += alpha_j p_j for the ring's pending directions, in the order of their steps.
static void ring_flush(saamg_state* S) {
    RingSlots rs{};
    rs.m = S->pend;
    for (int j = 0; j < S->pend; ++j) rs.slot[j] = ring_index(S, S->kdir - S->pend + j);
    if (S->mixed)
        cg_xring<float>(cg_op(S->H), S->x, (const float*)S->ring, S->scal, rs, S->s);
    else
        cg_xring<double>(cg_op(S->H), S->x, (const double*)S->ring, S->scal, rs, S->s);
    S->pend = 0;
}

// Partial sums written by the V-cycle's fused r . z (in the working precision).
static long pc_parts(const saamg_state* S) { return l0_dot_parts(S->H->l0, S->mixed ? 4 : 8); }

// pinned = false: no pinned host buffer and no event (the allocation-free solve); the
// scalars are read into the state itself and the host waits on the stream.
static void state_alloc(saamg_state* S, saamg_hierarchy* H, bool pinned = true) {
    S->H = H;
    S->mixed = H->opt.precision == SAAMG_MIXED;
    const long n = H->l0.nbox;
    S->x = (double*)dmalloc(8 * n);
    S->r = (double*)dmalloc(8 * n);
    S->ringf = cg_ring(H->l0);
    S->pw = S->mixed ? 4 : 8;
    if (S->ringf) {
        // a state that allocates nothing keeps 2 directions (flushed every other step)
        S->ringk = pinned ? cg_ring_len(n, S->pw, H->opt.cg_ring) : 2;
        S->ring = dmalloc((size_t)S->pw * S->ringk * n);
    } else {
        S->p = dmalloc(8 * n);
    }
    S->q = (double*)dmalloc(8 * n);
    S->bs = (double*)dmalloc(8 * n);
    S->z = dmalloc((S->mixed ? 4 : 8) * n);
    if (S->mixed) S->r32 = (float*)dmalloc(4 * n);
    // x, r, q, b~ (fp64); p, z and the fp32 copy of r
    S->bytes = 32L * n + (S->ringf ? (long)S->pw * S->ringk : 8) * n + 8L * n;  // z 8, or fp32 z and r32
    if (S->mixed) {
        S->vf.alloc(H);
        S->bytes += S->vf.bytes(H);
    } else {
        S->vd.alloc(H);
        S->bytes += S->vd.bytes(H);
    }
    S->npart = std::max<long>(l0_blocks(H->l0), 1);
    if (H->l0.wide)
        S->npart = std::max(S->npart, std::max(l0_wblocks(H->l0, 2), l0_wblocks(H->l0, 4)));
    S->part = (double*)dmalloc(sizeof(double) * 3 * S->npart);
    S->scal = (double*)dmalloc(sizeof(double) * S_NSLOTS);
    if (!pinned) {
        S->hscal = S->hbuf;
        return;
    }
    HIPCHECK(hipHostMalloc((void**)&S->hscal, sizeof(double) * S_NSLOTS, hipHostMallocDefault));
    HIPCHECK(hipEventCreateWithFlags(&S->ev, hipEventDisableTiming));
}

static void state_release(saamg_state* S) {
    for (double* p : {S->x, S->r, S->q, S->bs}) dfree(p);
    dfree(S->p);
    dfree(S->ring);
    dfree(S->z);
    dfree(S->r32);
    S->r32 = nullptr;
    S->vf.release();
    S->vd.release();
    dfree(S->part);
    dfree(S->scal);
    if (S->hscal && S->hscal != S->hbuf) (void)hipHostFree(S->hscal);
    if (S->ev) (void)hipEventDestroy(S->ev);
    S->x = S->r = S->q = S->bs = nullptr;
    S->z = S->p = nullptr;
    S->ring = nullptr;
    S->part = S->scal = S->hscal = nullptr;
    S->ev = nullptr;
}

static void read_scal(saamg_state* S) {
    HIPCHECK(hipMemcpyAsync(S->hscal, S->scal, sizeof(double) * S_NSLOTS, hipMemcpyDeviceToHost,
                            S->s));
    HIPCHECK(hipStreamSynchronize(S->s));
}

// z = M r and the partials of r . z.  The dot is taken with the residual the V-cycle
// reads (the fp32 copy in mixed precision, so r . z is the quadratic form of the applied
// preconditioner); a one-level hierarchy takes it with the fp64 residual.  With `skippable`
// the V-cycle's kernels honour the solve's skip flag (scal[S_SKIP]).
static void precond(saamg_state* S, bool skippable = true) {
    const saamg_hierarchy* H = S->H;
    VSkipScope vs(skippable ? S->scal + S_SKIP : nullptr);
    const double* fdot = H->n_levels == 1 ? S->r : nullptr;
    if (S->mixed)
        vcycle<float>(H, S->vf, 0, S->r32, (float*)S->z, fdot, S->part, S->s);
    else
        vcycle<double>(H, S->vd, 0, S->r, (double*)S->z, fdot, S->part, S->s);
}

// True residual b - A x into `dst`; returns ||dst||^2.
static double true_residual(saamg_state* S, double* dst) {
    cg_resid(cg_op(S->H), S->bs, S->x, dst, S->part, dst == S->r ? S->r32 : nullptr, S->s);
    finalize(S->part, cg_resid_parts(cg_op(S->H)), 2, S->scal, FIN_STORE, S_RT, S->s);
    read_scal(S);
    return S->hscal[S_RT];
}

static void state_start(saamg_state* S, const double* b, const double* x0) {
    const saamg_hierarchy* H = S->H;
    S->iter = 0;
    S->status = SAAMG_OK;
    S->done = 0;
    S->repl = 0;
    S->t0 = std::chrono::steady_clock::now();
    if (!x0 && cg_op(H).wide && (reinterpret_cast<uintptr_t>(b) & 15u) == 0) {
        // without an initial guess x = 0 and r = b~: one pass on 16-byte lanes
        w_cg_start(cg_op(H), b, S->bs, S->x, S->r, S->part, S->r32, S->s);
    } else {
        cg_init(cg_op(H), b, x0, S->bs, S->x, S->s);
        // without an initial guess x = 0 and r = b~ (no product with A)
        cg_resid(cg_op(H), S->bs, x0 ? S->x : nullptr, S->r, S->part, S->r32, S->s);
    }
    finalize(S->part, cg_resid_parts(cg_op(H)), 2, S->scal, FIN_STORE, S_RR, S->s);
    scal_start(S->scal, S->tol, S->s);
    S->kdir = 0;
    S->pend = 0;
    if (S->ringf)  // the direction the first step reads (times beta = 0)
        zero_fill((char*)S->ring + (size_t)S->pw * ring_index(S, -1) * H->l0.nbox,
                  (size_t)S->pw * H->l0.nbox, S->s);
    else
        zero_fill(S->p, 8 * H->l0.nbox, S->s);
    // the fused form carries A p in q; the ring form uses q only as scratch for a true
    // residual
    if (!S->ringf) zero_fill(S->q, 8 * H->l0.nbox, S->s);
    read_scal(S);
    const double rr = S->hscal[S_RR], bb = S->hscal[S_BB];
    S->bnorm = std::sqrt(bb);
    if (!std::isfinite(rr) || !std::isfinite(bb)) {
        S->status = SAAMG_NONFINITE;
        S->done = 1;
        S->rel_true = S->rel_rec = NAN;
        return;
    }
    if (bb == 0.0) {
        zero_fill(S->x, 8 * H->l0.nbox, S->s);
        S->done = 1;
        S->rel_true = S->rel_rec = 0.0;
        return;
    }
    const double rel = std::sqrt(rr) / S->bnorm;
    S->rel_true = S->rel_rec = rel;
    if (rel <= S->tol) {
        S->done = 1;
        return;
    }
    if (S->max_iter <= 0) {
        S->status = SAAMG_NOT_CONVERGED;
        S->done = 1;
        return;
    }
    precond(S);
    finalize(S->part, pc_parts(S), 1, S->scal, FIN_RHO_INIT, 0, S->s);
}

// Queue one PCG step plus the (speculative) preconditioner of the next one.
static void state_enqueue(saamg_state* S) {
    const saamg_hierarchy* H = S->H;
    const FineLevel& L = cg_op(H);
    if (S->ringf) {
        if (S->pend == S->ringk) ring_flush(S);  // the next direction overwrites the oldest
        if (S->mixed)
            cg_pdir<float>(L, (const float*)S->z, ring_at<float>(S, S->kdir - 1),
                           ring_at<float>(S, S->kdir), S->scal, S->part, S->s);
        else
            cg_pdir<double>(L, (const double*)S->z, ring_at<double>(S, S->kdir - 1),
                            ring_at<double>(S, S->kdir), S->scal, S->part, S->s);
    } else if (S->mixed)
        cg_pq<float>(L, (const float*)S->z, S->x, (double*)S->p, S->q, S->scal, S->part, S->s);
    else
        cg_pq<double>(L, (const double*)S->z, S->x, (double*)S->p, S->q, S->scal, S->part, S->s);
    finalize(S->part, cg_pq_parts(L, S->ringf, S->pw), 1, S->scal, FIN_ALPHA,
             S->ringf ? S_AR0 + ring_index(S, S->kdir) : 0, S->s);
    if (S->ringf) {
        if (S->mixed)
            cg_xr_dir<float>(L, ring_at<float>(S, S->kdir), S->r, S->r32, S->scal, S->part, S->s);
        else
            cg_xr_dir<double>(L, ring_at<double>(S, S->kdir), S->r, nullptr, S->scal, S->part,
                              S->s);
        S->kdir += 1;
        S->pend += 1;
    } else {
        cg_xr(L, S->r, S->q, S->scal, S->part, S->r32, S->s);
    }
    finalize(S->part, cg_xr_parts(L, S->ringf, S->pw), 1, S->scal, FIN_RR, 0, S->s);
    HIPCHECK(hipMemcpyAsync(S->hscal, S->scal, sizeof(double) * S_NSLOTS, hipMemcpyDeviceToHost,
                            S->s));
    if (S->ev) HIPCHECK(hipEventRecord(S->ev, S->s));
    S->inflight = true;
    precond(S);
    finalize(S->part, pc_parts(S), 1, S->scal, FIN_RHO, 0, S->s);
}

// The updates x still owes: the step length of the last step (applied by the next step's
// direction update in the fused form), or the ring's pending directions.  Needed before x
// is read.
static void flush_x(saamg_state* S) {
    if (S->ringf) {
        if (S->pend > 0) ring_flush(S);
        return;
    }
    cg_xflush<double>(cg_op(S->H), S->x, (const double*)S->p, S->scal, S->s);
    finalize(S->part, 1, 0, S->scal, FIN_XA_CLEAR, 0, S->s);
}

static void state_complete(saamg_state* S) {
    if (S->ev)
        HIPCHECK(hipEventSynchronize(S->ev));
    else
        HIPCHECK(hipStreamSynchronize(S->s));
    S->inflight = false;
    S->iter += 1;
    const double pq = S->hscal[S_PQ], rho = S->hscal[S_RHO], rr = S->hscal[S_RR];
    const double alpha = S->hscal[S_ALPHA];
    if (!std::isfinite(pq) || !std::isfinite(rho) || !std::isfinite(alpha)) {
        flush_x(S);
        S->status = SAAMG_NONFINITE;
        S->done = 1;
        S->rel_true = S->rel_rec = NAN;
        return;
    }
    if (pq <= 0.0 || rho <= 0.0) {
        flush_x(S);
        S->status = SAAMG_BREAKDOWN;
        S->done = 1;
        S->rel_true = std::sqrt(true_residual(S, S->q)) / S->bnorm;
        return;
    }
    if (!std::isfinite(rr)) {
        flush_x(S);
        S->status = SAAMG_NONFINITE;
        S->done = 1;
        S->rel_true = S->rel_rec = NAN;
        return;
    }
    S->rel_rec = std::sqrt(rr) / S->bnorm;
    if (S->rel_rec <= S->tol) {
        flush_x(S);
        const double rt = true_residual(S, S->r);
        S->rel_true = std::sqrt(rt) / S->bnorm;
        if (S->rel_true <= S->tol) {
            S->done = 1;
            return;
        }
        // continue from the true residual: redo the preconditioner on it (the restore
        // also clears the device's skip flag; the host copy follows)
        S->repl += 1;
        const long nb = pc_parts(S);
        finalize(S->part, nb, 0, S->scal, FIN_RESTORE_RHO, 0, S->s);
        precond(S);
        finalize(S->part, nb, 1, S->scal, FIN_RHO, 0, S->s);
        S->hscal[S_SKIP] = 0.0;
    }
    if (S->iter >= S->max_iter) {
        flush_x(S);
        S->status = SAAMG_NOT_CONVERGED;
        S->done = 1;
        S->rel_true = std::sqrt(true_residual(S, S->q)) / S->bnorm;
        return;
    }
    if (S->hscal[S_SKIP] != 0.0) {
        // the device skipped the queued V-cycle while the host goes on (the two tests
        // use the same expression, so only a rounding difference could cause this): redo
        // that step's preconditioner
        const long nb = pc_parts(S);
        finalize(S->part, nb, 0, S->scal, FIN_RESTORE_RHO, 0, S->s);
        precond(S);
        finalize(S->part, nb, 1, S->scal, FIN_RHO, 0, S->s);
    }
}

static void state_fill_result(const saamg_state* S, saamg_result* res) {
    if (!res) return;
    res->iterations = S->iter;
    res->status = S->status;
    res->replacements = S->repl;
    res->rel_res_true = S->rel_true;
    res->rel_res_recursive = S->rel_rec;
    res->t_solve_ms = S->t_ms;
}

// ------------------------------------------------------------------ setup

static long seg_count(int nx, int ny, int nz) { return (long)((nx + 63) / 64) * ny * nz; }

// Largest eigenvalue of the symmetric tridiagonal matrix with diagonal a[0..m-1] and
// off-diagonal b[0..m-2], by bisection on Sturm sequence counts.
static double tridiag_max_eig(const double* a, const double* b, int m) {
    double lo = a[0], hi = a[0];
    for (int i = 0; i < m; ++i) {
        const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(b[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    // number of eigenvalues below x = number of negative pivots of T - x I
    auto below = [&](double x) {
        int cnt = 0;
        double d = 1.0;
        for (int i = 0; i < m; ++i) {
            d = a[i] - x - (i > 0 ? b[i - 1] * b[i - 1] / d : 0.0);
            if (d == 0.0) d = -1e-300;
            if (d < 0.0) ++cnt;
        }
        return cnt;
    };
    for (int it = 0; it < 200 && hi - lo > 2e-16 * std::max(std::fabs(lo), std::fabs(hi)); ++it) {
        const double mid = 0.5 * (lo + hi);
        if (below(mid) == m)
            hi = mid;
        else
            lo = mid;
    }
    return 0.5 * (lo + hi);
}

// Upper end of the spectrum of D^-1 A on level l (the bound that the Chebyshev and the
// prolongator smoothers need, Section 3.2): the largest Ritz value of Lanczos steps in
// the D inner product on the symmetric part (A + A^T)/2, started from the SplitMix64
// vector of the box index.  The recurrence ends early when beta_k <= 1e-12 max|alpha|,
// and runs at most n steps on a level with n unknowns.
static double lanczos_lambda(saamg_hierarchy* H, int l, hipStream_t s) {
    const long n = (l == 0) ? H->l0.nbox : H->lc[l - 1].nstore;
    const long nb = (l == 0) ? l0_blocks(H->l0) : lc_blocks(H->lc[l - 1]);
    // level 0 on 16-byte lanes: the apply runs on the wide march (its own block count)
    const bool wide = (l == 0) && H->l0.wide;
    const long nb_apply = wide ? l0_wblocks(H->l0, 2) : nb;
    const long n_unk = (l == 0) ? H->l0.n_unknowns : H->lc[l - 1].n_unknowns;
    const int K = (int)std::min<long>(H->opt.eig_iters, n_unk);
    Tmp t_cur(8 * n), t_prev(8 * n), t_u(8 * n), t_part(sizeof(double) * std::max(nb, nb_apply)),
        t_scal(sizeof(double) * (S_NSLOTS + 2 * K));
    double* cur = t_cur.as<double>();
    double* prev = t_prev.as<double>();
    double* u = t_u.as<double>();
    double* part = t_part.as<double>();
    double* scal = t_scal.as<double>();
    if (l == 0)
        l0_lz_start(H->l0, cur, part, s);
    else
        lc_lz_start(H->lc[l - 1], cur, part, s);
    finalize(part, nb, 1, scal, FIN_NORM, 0, s);
    for (int k = 0; k < K; ++k) {
        if (wide)
            w_lz_apply(H->l0, H->sym, cur, scal, u, part, s);
        else if (l == 0)
            l0_lz_apply(H->l0, H->sym, cur, scal, u, part, s);
        else
            lc_lz_apply(H->lc[l - 1], cur, scal, u, part, s);
        finalize(part, nb_apply, 1, scal, FIN_LZ_ALPHA, S_NSLOTS + k, s);
        if (l == 0)
            l0_lz_update(H->l0, u, cur, prev, scal, part, s);
        else
            lc_lz_update(H->lc[l - 1], u, cur, prev, scal, part, s);
        finalize(part, nb, 1, scal, FIN_LZ_BETA, S_NSLOTS + K + k, s);
        std::swap(cur, prev);
    }
    std::vector<double> ab(2 * K);
    HIPCHECK(hipMemcpyAsync(ab.data(), scal + S_NSLOTS, sizeof(double) * 2 * K,
                            hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    const double* alpha = ab.data();
    const double* beta = ab.data() + K;
    int m = 0;
    double amax = 0.0;
    while (m < K) {
        amax = std::max(amax, std::fabs(alpha[m]));
        ++m;
        if (beta[m - 1] <= 1e-12 * amax) break;
    }
    for (int k = 0; k < m; ++k)
        if (!std::isfinite(alpha[k]) || !std::isfinite(beta[k])) return NAN;
    return tridiag_max_eig(alpha, beta, m);
}

static void free_coarse(CoarseLevel& C);

static CoarseLevel make_coarse(int fmx, int fmy, int fmz, int sym) {
    CoarseLevel C;
    C.mx = (fmx + 2) / 3;
    C.my = (fmy + 2) / 3;
    C.mz = (fmz + 2) / 3;
    C.sx = C.mx + 2;
    C.sy = C.my + 2;
    C.sz = C.mz + 2;
    C.sxy = (long)C.sx * C.sy;
    C.nstore = C.sxy * C.sz;
    C.sym = sym;
    // the coefficient arrays (27, or the 14 of offsets k >= 13 on symmetric levels) and
    // 1/diag in one allocation, each array 256-byte aligned: one zero fill for all of them
    const long stride = (C.nstore + 31) & ~31L;
    const int na = sym ? 14 : 27;
    C.block64 = (double*)dmalloc(8 * stride * (na + 1));
    int j = 0;
    for (int k = 0; k < 27; ++k)
        if (!sym || k >= 13) C.coef64[k] = C.block64 + stride * j++;
    C.invD64 = C.block64 + stride * j;
    return C;
}

static void free_coarse(CoarseLevel& C) {
    dfree(C.block64);  // the coef64 arrays and invD64
    C.block64 = nullptr;
    for (int k = 0; k < 27; ++k) C.coef64[k] = nullptr;
    for (void* p : {(void*)C.invD32, (void*)C.slot, (void*)C.tab64, (void*)C.tab32,
                    (void*)C.slotT, (void*)C.tabT64, (void*)C.tabT32})
        dfree(p);
    C.invD64 = nullptr;
    C.invD32 = nullptr;
    C.slot = C.slotT = nullptr;
    C.tab64 = C.tabT64 = nullptr;
    C.tab32 = C.tabT32 = nullptr;
    C.tab_cap = C.n_tab = C.tabT_cap = C.n_tabT = 0;
}

static int64_t coarse_bytes(const CoarseLevel& C, bool mixed) {
    const int na = C.sym ? 14 : 27;
    return (int64_t)(na + 1) * ((C.nstore + 31) & ~31L) * 8 + 4L * C.nstore * (C.sym ? 1 : 2) +
           (mixed ? 4L * C.nstore : 0) + (long)kLcRow * (C.tab_cap + C.tabT_cap) * (mixed ? 12 : 8);
}

static void validate_options(const saamg_options& o) {
    if (o.precision != SAAMG_FP64 && o.precision != SAAMG_MIXED)
        throw ApiError{SAAMG_INVALID_ARG, "precision must be SAAMG_FP64 or SAAMG_MIXED"};
    if (o.max_levels < 1 || o.max_levels > SAAMG_MAX_LEVELS)
        throw ApiError{SAAMG_INVALID_ARG, "max_levels must be in 1..16"};
    if (o.max_coarse < 1 || o.max_coarse > 8000)
        throw ApiError{SAAMG_INVALID_ARG, "max_coarse must be in 1..8000"};
    if (o.cheb_degree < 1 || o.cheb_degree > 8)
        throw ApiError{SAAMG_INVALID_ARG, "cheb_degree must be in 1..8"};
    if (!(o.cheb_ratio > 1.0) || !(o.cheb_boost > 0.0) || !(o.omega_scale > 0.0))
        throw ApiError{SAAMG_INVALID_ARG, "cheb_ratio must exceed 1; boost and omega_scale > 0"};
    if (o.eig_iters < 1 || o.eig_iters > 1000)
        throw ApiError{SAAMG_INVALID_ARG, "eig_iters must be in 1..1000"};
    if (o.coarse_solver != SAAMG_COARSE_DIRECT && o.coarse_solver != SAAMG_COARSE_GS)
        throw ApiError{SAAMG_INVALID_ARG, "coarse_solver must be SAAMG_COARSE_DIRECT or _GS"};
    if (o.coarse_sweeps < 1 || o.coarse_sweeps > 100)
        throw ApiError{SAAMG_INVALID_ARG, "coarse_sweeps must be in 1..100"};
    // the march loads one mask word per plane of a block and its two halo planes into
    // the lanes of a wavefront, so a block holds at most 32 planes
    if (o.l0_planes != 0 && (o.l0_planes < 2 || o.l0_planes > 32 || (o.l0_planes & (o.l0_planes - 1))))
        throw ApiError{SAAMG_INVALID_ARG, "l0_planes must be 0 or a power of two in 2..32"};
    if (o.l0_tile_x != 0 && o.l0_tile_x != 1 && o.l0_tile_x != 2 && o.l0_tile_x != 4)
        throw ApiError{SAAMG_INVALID_ARG, "l0_tile_x must be 0, 1, 2 or 4"};
    if ((o.alloc == nullptr) != (o.free == nullptr))
        throw ApiError{SAAMG_INVALID_ARG, "alloc and free must both be set or both be NULL"};
    if (o.cg_ring != 0 && (o.cg_ring < 2 || o.cg_ring > kCgRing))
        throw ApiError{SAAMG_INVALID_ARG, "cg_ring must be 0 (automatic) or 2..32"};
    if (o.l0_wide < 0 || o.l0_wide > 2)
        throw ApiError{SAAMG_INVALID_ARG, "l0_wide must be 0, 1 or 2"};
}

struct DeviceDomain {
    uint8_t* mask = nullptr;
    int32_t* nwidx = nullptr;
    int64_t* nwnodes = nullptr;
    double* nwfrac = nullptr;
    DeviceDomain(const saamg_domain* dom, const DomainPrep& D, long nbox, hipStream_t s) {
        try {
            mask = (uint8_t*)dmalloc(nbox);
            nwidx = (int32_t*)dmalloc(4 * nbox);
            nwnodes = (int64_t*)dmalloc(8 * std::max<size_t>(D.nw_nodes.size(), 1));
            nwfrac = (double*)dmalloc(8 * std::max<size_t>(D.nw_frac.size(), 1));
            // uploads and the fill are queued on s, ordered before the kernels that read
            // them; the host arrays outlive the setup's next synchronisation of s
            HIPCHECK(hipMemcpyAsync(mask, dom->mask, nbox, hipMemcpyHostToDevice, s));
            HIPCHECK(hipMemsetAsync(nwidx, 0xff, 4 * nbox, s));
            if (!D.nw_nodes.empty()) {
                HIPCHECK(hipMemcpyAsync(nwnodes, D.nw_nodes.data(), 8 * D.nw_nodes.size(),
                                        hipMemcpyHostToDevice, s));
                HIPCHECK(hipMemcpyAsync(nwfrac, D.nw_frac.data(), 8 * D.nw_frac.size(),
                                        hipMemcpyHostToDevice, s));
            }
            l0_scatter_nwidx(nwidx, nwnodes, (long)D.nw_nodes.size(), s);
            HIPCHECK(hipStreamSynchronize(s));
        } catch (...) {
            release();
            throw;
        }
    }
    void release() {
        for (void* p : {(void*)mask, (void*)nwidx, (void*)nwnodes, (void*)nwfrac}) dfree(p);
        mask = nullptr;
        nwidx = nullptr;
        nwnodes = nullptr;
        nwfrac = nullptr;
    }
    ~DeviceDomain() { release(); }
};

// Level-0 numbers from the spacings, the Robin parameter and the near-wall fractions:
// stencil weights of regular rows, the irregular rows' table and the scaling sigma.
static void fine_numbers(FineLevel& L, const saamg_domain* dom, const DeviceDomain& dd, int variant,
                         hipStream_t s) {
    L.h[0] = dom->hx;
    L.h[1] = dom->hy;
    L.h[2] = dom->hz;
    L.robin_d = dom->robin_d;
    const double ih2[3] = {1.0 / (L.h[0] * L.h[0]), 1.0 / (L.h[1] * L.h[1]),
                           1.0 / (L.h[2] * L.h[2])};
    const double sigma0 = 1.0 / std::sqrt(2.0 * ih2[0] + 2.0 * ih2[1] + 2.0 * ih2[2]);
    for (int a = 0; a < 3; ++a) L.c64[a] = -(sigma0 * (1.0 * ih2[a])) * sigma0;
    const long nr = std::max<long>(L.n_irr, 1);
    Tmp full64(8 * 16 * nr), full32(4 * 16 * nr);
    l0_build_table(L, dd.mask, dd.nwidx, dd.nwfrac, variant, sigma0, full64.as<double>(),
                   full32.as<float>(), s);
    l0_dedup_table(L, full64.as<double>(), full32.as<float>(), s);
}

// Smoother and transfer parameters of level l from its operator (Section 3.2).
static LevelParams level_params(saamg_hierarchy* H, int l, hipStream_t s) {
    const saamg_options& o = H->opt;
    LevelParams P;
    P.lam = lanczos_lambda(H, l, s);
    if (!(P.lam > 0) || !std::isfinite(P.lam))
        throw ApiError{SAAMG_HIP_ERROR, "spectral estimate failed on level " + std::to_string(l)};
    P.lam_hi = o.cheb_boost * P.lam;
    P.omega = o.omega_scale / P.lam;
    P.cheb = cheb_coefficients(P.lam_hi, o.cheb_ratio, o.cheb_degree);
    return P;
}

// Galerkin operator of level l+1 into C, its inverse diagonal, and the number of coarse
// unknowns (aggregates holding at least one unknown); `cnt_out` (nullable) receives the
// per-64 counts, which the caller frees.
static int64_t galerkin(saamg_hierarchy* H, int l, CoarseLevel& C, double omega,
                        int32_t** cnt_out, hipStream_t s) {
    if (l == 0)
        rap_from_l0(H->l0, C, omega, s);
    else
        rap_from_lc(H->lc[l - 1], C, omega, s);
    const long nb = (C.nstore + 255) / 256;
    int32_t* cnt = (int32_t*)dmalloc(4 * 4 * nb);
    int64_t nc = 0;
    try {
        lc_finish(C, cnt, s);
        lc_compress(C, s);
        Tmp tot(8 * scan_words(4 * nb));
        exclusive_scan(cnt, nullptr, 4 * nb, tot.as<int64_t>(), s);
        HIPCHECK(hipMemcpyAsync(&nc, tot.p, 8, hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
    } catch (...) {
        (void)hipStreamSynchronize(s);
        dfree(cnt);
        throw;
    }
    if (cnt_out)
        *cnt_out = cnt;
    else
        dfree(cnt);
    return nc;
}

// Coarsest-level solver: Gauss-Seidel sweeps need nothing beyond the stored operator;
// the direct solver holds the explicit fp64 inverse (allocated on first use).
static void build_coarse_solver(saamg_hierarchy* H, hipStream_t s) {
    if (H->opt.coarse_solver == SAAMG_COARSE_GS) {
        if (H->lc.back().nstore > kGsMax)
            throw ApiError{SAAMG_INVALID_ARG,
                           "coarsest level too large for the Gauss-Seidel solver; lower max_coarse"};
        return;
    }
    const int nL = H->nL;
    const long nstore = (H->n_levels == 1) ? H->l0.nbox : H->lc.back().nstore;
    int32_t* cmap = (int32_t*)dmalloc(4 * nstore);
    try {
        HIPCHECK(hipMemsetAsync(cmap, 0xff, 4 * nstore, s));
        fill_cmap(cmap, H->cidx, nL, s);
        if (!H->Ainv) {
            H->Ainv = (double*)dmalloc(8L * nL * nL);
            H->bytes += 8L * nL * nL + 8L * nL;
        } else {
            // the assembly writes the nonzero couplings only
            HIPCHECK(hipMemsetAsync(H->Ainv, 0, 8L * nL * nL, s));
        }
        if (H->n_levels == 1)
            dense_from_l0(H->l0, H->cidx, cmap, nL, H->Ainv, s);
        else
            dense_from_lc(H->lc.back(), H->cidx, cmap, nL, H->Ainv, s);
        dense_invert(H->Ainv, nL, s);
        HIPCHECK(hipStreamSynchronize(s));
    } catch (...) {
        dfree(cmap);
        throw;
    }
    dfree(cmap);
}

// fp32 copies of the coarse operators for the mixed-precision V-cycle (allocated on
// first use).
static void coarse_fp32(saamg_hierarchy* H, hipStream_t s) {
    if (H->opt.precision != SAAMG_MIXED) return;
    for (auto& C : H->lc) {
        if (!C.tab32) C.tab32 = (float*)dmalloc(4 * kLcRow * C.tab_cap);
        if (C.tabT64 && !C.tabT32) C.tabT32 = (float*)dmalloc(4 * kLcRow * C.tabT_cap);
        if (!C.invD32) C.invD32 = (float*)dmalloc(4 * C.nstore);
        lc_to_fp32(C, s);
    }
    HIPCHECK(hipStreamSynchronize(s));
}

static saamg_hierarchy* setup_impl(const saamg_domain* dom, int variant, const saamg_options* opt,
                                   hipStream_t s) {
    auto t0 = std::chrono::steady_clock::now();
    const DomainPrep D = prepare_domain(dom, variant);
    const double t_host = ms_since(t0);
    saamg_options o;
    if (opt)
        o = *opt;
    else
        saamg_default_options(&o);
    validate_options(o);
    const int nx = dom->nx, ny = dom->ny, nz = dom->nz;
    const long nxy = (long)nx * ny, nbox = nxy * nz;

    saamg_hierarchy* H = new saamg_hierarchy();
    H->mem.alloc = o.alloc;
    H->mem.free = o.free;
    H->mem.ctx = o.alloc_ctx;
    try {
        HIPCHECK(hipGetDevice(&H->device));
        H->variant = variant;
        H->opt = o;
        H->sym = variant != SAAMG_VARIANT_QUAD;
        FineLevel& L = H->l0;
        L.nx = nx;
        L.ny = ny;
        L.nz = nz;
        L.nsegx = (nx + 63) / 64;
        L.nxy = nxy;
        L.nbox = nbox;
        L.nseg = seg_count(nx, ny, nz);
        if (o.l0_tile_x > L.nsegx)
            throw ApiError{SAAMG_INVALID_ARG, "l0_tile_x exceeds the 64-node segments of a line"};
        L.tx = o.l0_tile_x ? o.l0_tile_x : l0_tile_x(L.nsegx);
        L.zb = o.l0_planes ? o.l0_planes : l0_choose_zb(L.tx, L.nsegx, ny, nz);
        if (o.l0_wide == 2 && nx % 4 != 0)
            throw ApiError{SAAMG_INVALID_ARG, "l0_wide = 2 needs nx to be a multiple of 4"};
        L.wide = o.l0_wide == 2 ? 1 : (o.l0_wide == 1 ? 0 : (int)l0_wide_default(nx));
        L.wzb[0] = l0_wide_zb(L, 2, o.l0_planes);
        L.wzb[1] = l0_wide_zb(L, 4, o.l0_planes);
        L.unk = (uint64_t*)dmalloc(8 * L.nseg);
        L.irr = (uint64_t*)dmalloc(8 * L.nseg);
        L.base = (int32_t*)dmalloc(4 * L.nseg);
        L.base_full = (int32_t*)dmalloc(4 * L.nseg);
        L.sigma = (double*)dmalloc(8 * nbox);

        // segment masks of unknowns and irregular rows, table slots
        DeviceDomain dd(dom, D, nbox, s);
        int64_t tots[2];
        {
            // two totals: the second scan's total sits in the first one's scratch, which it
            // no longer needs when the second scan (queued after it) writes there
            Tmp cnt_irr(4 * L.nseg), cnt_unk(4 * L.nseg), d_tot(8 * (1 + scan_words(L.nseg)));
            l0_build_masks(L, dd.mask, dd.nwidx, cnt_irr.as<int32_t>(), cnt_unk.as<int32_t>(), s);
            exclusive_scan(cnt_irr.as<int32_t>(), L.base_full, L.nseg, d_tot.as<int64_t>(), s);
            exclusive_scan(cnt_unk.as<int32_t>(), nullptr, L.nseg, d_tot.as<int64_t>() + 1, s);
            HIPCHECK(hipMemcpyAsync(tots, d_tot.p, 16, hipMemcpyDeviceToHost, s));
            HIPCHECK(hipStreamSynchronize(s));
        }
        L.n_irr = tots[0];
        L.n_unknowns = tots[1];
        fine_numbers(L, dom, dd, variant, s);
        dd.release();
        H->bytes = 24L * L.nseg + 8L * nbox + 12L * 16 * L.n_tab;
        H->t_phase_ms[0] = t_host;
        H->t_phase_ms[1] = ms_since(t0) - t_host;

        // hierarchy (Section 3.2): coarsen until at most max_coarse unknowns
        long n_cur = L.n_unknowns;
        int fmx = nx, fmy = ny, fmz = nz;
        H->n_levels = 1;
        while (n_cur > o.max_coarse && H->n_levels < o.max_levels) {
            const int l = H->n_levels - 1;
            auto tl = std::chrono::steady_clock::now();
            const LevelParams P = level_params(H, l, s);
            H->t_phase_ms[2] += ms_since(tl);
            tl = std::chrono::steady_clock::now();
            CoarseLevel C = make_coarse(fmx, fmy, fmz, H->sym);
            int32_t* cnt = nullptr;
            int64_t nc = 0;
            try {
                nc = galerkin(H, l, C, P.omega, &cnt, s);
                H->t_phase_ms[3] += ms_since(tl);
            } catch (...) {
                free_coarse(C);
                throw;
            }
            if (nc >= n_cur) {
                // the aggregates no longer reduce the unknowns: the level built last is
                // the coarsest (as the oracle's setup does)
                dfree(cnt);
                free_coarse(C);
                break;
            }
            C.n_unknowns = nc;
            if (nc <= o.max_coarse || H->n_levels + 1 == o.max_levels) {
                // coarsest level: collect its unknowns
                if (nc > 8000) {
                    dfree(cnt);
                    free_coarse(C);
                    throw ApiError{SAAMG_INVALID_ARG, "coarsest level too large"};
                }
                H->nL = (int)nc;
                H->cidx = (long*)dmalloc(8 * nc);
                lc_unknown_list(C, H->cidx, cnt, s);
            }
            dfree(cnt);
            H->par.push_back(P);
            H->lc.push_back(C);
            H->bytes += coarse_bytes(C, o.precision == SAAMG_MIXED);
            H->n_levels += 1;
            n_cur = nc;
            fmx = C.mx;
            fmy = C.my;
            fmz = C.mz;
        }
        if (H->n_levels == 1) {
            if (L.n_unknowns > 8000)
                throw ApiError{SAAMG_INVALID_ARG, "single-level hierarchy too large for a direct solve"};
            H->nL = (int)L.n_unknowns;
            H->cidx = (long*)dmalloc(8 * H->nL);
            l0_unknown_list(L, H->cidx, s);
        } else if (!H->cidx) {
            // coarsening stopped on a level that was not marked coarsest when it was built
            CoarseLevel& C = H->lc.back();
            if (C.n_unknowns > 8000)
                throw ApiError{SAAMG_INVALID_ARG,
                               "coarsening stalled above 8000 unknowns; the coarsest level is too "
                               "large for a direct solve"};
            const long nb = (C.nstore + 255) / 256;
            Tmp cnt(4 * 4 * nb);
            lc_finish(C, cnt.as<int32_t>(), s);  // recomputes 1/diag (same values) and the counts
            H->nL = (int)C.n_unknowns;
            H->cidx = (long*)dmalloc(8 * H->nL);
            lc_unknown_list(C, H->cidx, cnt.as<int32_t>(), s);
        }
        // Gauss-Seidel coarse solves need a coarse level to run on
        if (o.coarse_solver == SAAMG_COARSE_GS && H->n_levels == 1)
            H->opt.coarse_solver = SAAMG_COARSE_DIRECT;
        auto tc = std::chrono::steady_clock::now();
        build_coarse_solver(H, s);
        H->t_phase_ms[4] = ms_since(tc);
        tc = std::chrono::steady_clock::now();
        coarse_fp32(H, s);
        H->t_phase_ms[5] = ms_since(tc);
    } catch (...) {
        saamg_destroy(H);
        throw;
    }
    H->t_setup_ms = ms_since(t0);
    return H;
}

// Checks shared by the re-setups of H for a new domain: the box, the end condition kind
// and no live solve state.
static DomainPrep check_resetup(const saamg_hierarchy* H, const saamg_domain* dom) {
    const FineLevel& L = H->l0;
    if (dom && dom->mask && (dom->nx != L.nx || dom->ny != L.ny || dom->nz != L.nz))
        throw ApiError{SAAMG_INVALID_ARG, "the domain's box differs from the hierarchy's"};
    DomainPrep D = prepare_domain(dom, H->variant, false);
    if ((dom->robin_d > 0.0) != (L.robin_d > 0.0))
        throw ApiError{SAAMG_INVALID_ARG, "the end condition kind (open or closed) differs"};
    if (H->live_states > 0)
        throw ApiError{SAAMG_INVALID_ARG, "solve states of this hierarchy still exist"};
    return D;
}

// The new domain's segment masks (unknowns and near-wall rows) must equal H's.
static void check_same_rows(const saamg_hierarchy* H, const DeviceDomain& dd, hipStream_t s) {
    const FineLevel& L = H->l0;
    FineLevel T = L;
    Tmp unk(8 * L.nseg), irr(8 * L.nseg), c1(4 * L.nseg), c2(4 * L.nseg);
    T.unk = unk.as<uint64_t>();
    T.irr = irr.as<uint64_t>();
    l0_build_masks(T, dd.mask, dd.nwidx, c1.as<int32_t>(), c2.as<int32_t>(), s);
    if (!l0_same_masks(L, T.unk, T.irr, s))
        throw ApiError{SAAMG_INVALID_ARG,
                       "the domain's unknowns or near-wall rows differ from the hierarchy's"};
}

// End a reuse of the preconditioner: the CG iteration goes back to the hierarchy's own
// level-0 operator.
static void drop_operator(saamg_hierarchy* H) {
    if (!H->op) return;
    for (void* p : {(void*)H->op->tab64, (void*)H->op->tab32, (void*)H->op->sigma,
                    (void*)H->op->base})
        dfree(p);
    H->bytes -= 8L * H->op->nbox + 4L * H->op->nseg + 12L * 16 * H->op->n_tab;
    delete H->op;
    H->op = nullptr;
}

// Numeric-only re-setup on the aggregates, storage and buffers of H (Section 5.2, reuse of
// the aggregation hierarchy): the domain must have H's box, unknowns, near-wall rows and
// end condition kind; every number is recomputed.  H is unchanged when a check fails.
static void refresh_impl(saamg_hierarchy* H, const saamg_domain* dom, hipStream_t s) {
    auto t0 = std::chrono::steady_clock::now();
    FineLevel& L = H->l0;
    const DomainPrep D = check_resetup(H, dom);
    DeviceDomain dd(dom, D, L.nbox, s);
    check_same_rows(H, dd, s);
    // from here on H changes; a failure leaves it unusable (destroy it)
    drop_operator(H);
    H->bytes -= 12L * 16 * L.n_tab;
    fine_numbers(L, dom, dd, H->variant, s);
    H->bytes += 12L * 16 * L.n_tab;
    dd.release();
    for (int l = 0; l + 1 < H->n_levels; ++l) {
        H->par[l] = level_params(H, l, s);
        CoarseLevel& C = H->lc[l];
        H->bytes -= coarse_bytes(C, H->opt.precision == SAAMG_MIXED);
        const int64_t nc = galerkin(H, l, C, H->par[l].omega, nullptr, s);
        H->bytes += coarse_bytes(C, H->opt.precision == SAAMG_MIXED);
        if (nc != C.n_unknowns)
            throw ApiError{SAAMG_HIP_ERROR, "coarse level " + std::to_string(l + 1) +
                                                " changed its unknowns; destroy the hierarchy"};
    }
    build_coarse_solver(H, s);
    coarse_fp32(H, s);
    H->t_refresh_ms = ms_since(t0);
}

// Reuse of the preconditioner (Section 5.2): the CG iteration takes the level-0 operator
// (stencil weights, wall rows, scaling) of dom; the V-cycle keeps everything it had.
static void set_operator_impl(saamg_hierarchy* H, const saamg_domain* dom, hipStream_t s) {
    const FineLevel& L = H->l0;
    const DomainPrep D = check_resetup(H, dom);
    DeviceDomain dd(dom, D, L.nbox, s);
    check_same_rows(H, dd, s);
    if (!H->op) {
        // shares the segment masks and the rows' full slots; its own de-duplicated slots
        // and table (fine_numbers)
        FineLevel* op = new FineLevel(L);
        op->tab64 = nullptr;
        op->tab32 = nullptr;
        op->sigma = nullptr;
        op->base = nullptr;
        try {
            op->base = (int32_t*)dmalloc(4 * L.nseg);
            op->sigma = (double*)dmalloc(8 * L.nbox);
        } catch (...) {
            for (void* p : {(void*)op->base, (void*)op->sigma}) dfree(p);
            delete op;
            throw;
        }
        H->op = op;
        H->bytes += 8L * L.nbox + 4L * L.nseg;
    }
    H->bytes -= 12L * 16 * H->op->n_tab;
    fine_numbers(*H->op, dom, dd, H->variant, s);
    H->bytes += 12L * 16 * H->op->n_tab;
}

template <class F>
static int guarded(F&& f) {
    try {
        g_err.clear();
        return f();
    } catch (const ApiError& e) {
        g_err = e.msg;
        return e.status;
    } catch (const HipError& e) {
        g_err = std::string("HIP error ") + hipGetErrorString(e.e) + " in " + e.where;
        return SAAMG_HIP_ERROR;
    } catch (const std::bad_alloc&) {
        g_err = "host allocation failed";
        return SAAMG_NOMEM;
    } catch (const std::exception& e) {
        g_err = e.what();
        return SAAMG_INVALID_ARG;
    }
}

// Host logical <-> device storage helpers for the component entry points.
static long level_nstore(const saamg_hierarchy* H, int l) {
    return l == 0 ? H->l0.nbox : H->lc[l - 1].nstore;
}
static void level_dims(const saamg_hierarchy* H, int l, int* mx, int* my, int* mz) {
    if (l == 0) {
        *mx = H->l0.nx;
        *my = H->l0.ny;
        *mz = H->l0.nz;
    } else {
        *mx = H->lc[l - 1].mx;
        *my = H->lc[l - 1].my;
        *mz = H->lc[l - 1].mz;
    }
}
static long storage_index(const saamg_hierarchy* H, int l, int x, int y, int z) {
    if (l == 0) return x + (long)H->l0.nx * y + H->l0.nxy * z;
    const CoarseLevel& C = H->lc[l - 1];
    return (x + 1) + (long)C.sx * (y + 1) + C.sxy * (z + 1);
}

template <typename T>
static T* upload_level(const saamg_hierarchy* H, int l, const double* h) {
    int mx, my, mz;
    level_dims(H, l, &mx, &my, &mz);
    std::vector<T> buf(level_nstore(H, l), (T)0);
    // level 0: entries at nodes that are not unknowns are ignored (the kernels expect 0)
    std::vector<uint64_t> unk;
    if (l == 0) {
        unk.resize(H->l0.nseg);
        HIPCHECK(hipMemcpy(unk.data(), H->l0.unk, 8 * H->l0.nseg, hipMemcpyDeviceToHost));
    }
    for (int z = 0; z < mz; ++z)
        for (int y = 0; y < my; ++y)
            for (int x = 0; x < mx; ++x) {
                if (l == 0 &&
                    !((unk[((long)z * my + y) * H->l0.nsegx + (x >> 6)] >> (x & 63)) & 1ull))
                    continue;
                buf[storage_index(H, l, x, y, z)] = (T)h[x + (long)mx * (y + (long)my * z)];
            }
    T* d = (T*)dmalloc(sizeof(T) * buf.size());
    HIPCHECK(hipMemcpy(d, buf.data(), sizeof(T) * buf.size(), hipMemcpyHostToDevice));
    return d;
}

template <typename T>
static void download_level(const saamg_hierarchy* H, int l, const T* d, double* h) {
    int mx, my, mz;
    level_dims(H, l, &mx, &my, &mz);
    std::vector<T> buf(level_nstore(H, l));
    HIPCHECK(hipMemcpy(buf.data(), d, sizeof(T) * buf.size(), hipMemcpyDeviceToHost));
    for (int z = 0; z < mz; ++z)
        for (int y = 0; y < my; ++y)
            for (int x = 0; x < mx; ++x)
                h[x + (long)mx * (y + (long)my * z)] = (double)buf[storage_index(H, l, x, y, z)];
}

template <typename T>
static void level_apply_impl(saamg_hierarchy* H, int l, int op, const double* hin, double* hout) {
    hipStream_t s = nullptr;
    const int lin = (op == SAAMG_OP_PROLONG) ? l + 1 : l;
    const int lout = (op == SAAMG_OP_RESTRICT) ? l + 1 : l;
    T* din = upload_level<T>(H, lin, hin);
    T* dout = (T*)dmalloc(sizeof(T) * level_nstore(H, lout));
    T* tmp = (T*)dmalloc(sizeof(T) * level_nstore(H, l));
    switch (op) {
        case SAAMG_OP_APPLY:
        case SAAMG_OP_APPLY_T:
            if (l == 0)
                l0_apply<T>(H->l0, op == SAAMG_OP_APPLY_T, din, dout, s);
            else
                lc_apply<T>(H->lc[l - 1], op == SAAMG_OP_APPLY_T, din, dout, s);
            break;
        case SAAMG_OP_PRESMOOTH: {
            const ChebCoef& c = H->par[l].cheb;
            T* x = dout;
            T* other = tmp;
            T* d = (T*)dmalloc(sizeof(T) * level_nstore(H, l));
            auto step = [&](int mode, const T* xi, const T* di, T* xo, T* dd, double c1, double c2) {
                if (l == 0)
                    l0_cheb<T, T>(H->l0, mode, din, xi, di, xo, dd, c1, c2, c.c2[0], nullptr,
                                  nullptr, s);
                else
                    lc_cheb<T>(H->lc[l - 1], mode, din, xi, di, xo, dd, c1, c2, c.c2[0], s);
            };
            if (c.degree == 1) {
                step(CHEB_ZERO1, nullptr, nullptr, x, nullptr, 0, 0);
            } else {
                if (l > 0) lc_dscale<T>(H->lc[l - 1], din, other, s);  // D^-1 f
                step(CHEB_ZERO2, l > 0 ? other : nullptr, nullptr, x, d, c.c1[1], c.c2[1]);
                for (int k = 2; k < c.degree; ++k) {
                    step(CHEB_NEXT, x, d, other, d, c.c1[k], c.c2[k]);
                    std::swap(x, other);
                }
            }
            if (x != dout) HIPCHECK(hipMemcpy(dout, x, sizeof(T) * level_nstore(H, l), hipMemcpyDeviceToDevice));
            HIPCHECK(hipDeviceSynchronize());
            dfree(d);
            break;
        }
        case SAAMG_OP_RESTRICT:
            if (l == 0) {
                l0_restrict<T>(H->l0, H->lc[0], din, tmp, dout, nullptr, H->par[0].omega, s);
            } else {
                lc_dscale<T>(H->lc[l - 1], din, tmp, s);
                lc_restrict<T>(H->lc[l - 1], H->lc[l], din, tmp, dout, nullptr, H->par[l].omega,
                               s);
            }
            break;
        case SAAMG_OP_PROLONG:
            if (l == 0)
                l0_prolong<T>(H->l0, H->lc[0], din, dout, H->par[0].omega, s);
            else
                lc_prolong<T>(H->lc[l - 1], H->lc[l], din, dout, H->par[l].omega, s);
            break;
    }
    HIPCHECK(hipDeviceSynchronize());
    download_level<T>(H, lout, dout, hout);
    dfree(din);
    dfree(dout);
    dfree(tmp);
}

}  // namespace saamg

// ================================================================== C interface

extern "C" {

const char* saamg_last_error(void) { return saamg::g_err.c_str(); }

void saamg_default_options(saamg_options* o) {
    if (!o) return;
    o->precision = SAAMG_FP64;
    o->max_levels = 10;
    o->max_coarse = 1000;
    o->cheb_degree = 2;
    o->cheb_ratio = 10.0;
    o->cheb_boost = 1.1;
    o->eig_iters = 15;
    o->omega_scale = 4.0 / 3.0;
    o->coarse_solver = SAAMG_COARSE_DIRECT;
    o->coarse_sweeps = 3;
    o->l0_planes = 0;
    o->l0_tile_x = 0;
    o->l0_wide = 0;
    o->cg_ring = 0;
    o->alloc = nullptr;
    o->free = nullptr;
    o->alloc_ctx = nullptr;
}

int saamg_setup(const saamg_domain* dom, int variant, const saamg_options* opt, void* stream,
                saamg_hierarchy** out) {
    return guarded([&] {
        if (!out) throw ApiError{SAAMG_INVALID_ARG, "out is NULL"};
        *out = nullptr;
        MemCtx m;
        if (opt) {
            m.alloc = opt->alloc;
            m.free = opt->free;
            m.ctx = opt->alloc_ctx;
        }
        MemScope ms(m, (hipStream_t)stream);
        *out = setup_impl(dom, variant, opt, (hipStream_t)stream);
        return (int)SAAMG_OK;
    });
}

int saamg_set_operator(saamg_hierarchy* H, const saamg_domain* dom, void* stream) {
    return guarded([&] {
        if (!H) throw ApiError{SAAMG_INVALID_ARG, "hierarchy is NULL"};
        HIPCHECK(hipSetDevice(H->device));
        MemScope ms(H->mem, (hipStream_t)stream);
        set_operator_impl(H, dom, (hipStream_t)stream);
        return (int)SAAMG_OK;
    });
}

int saamg_refresh(saamg_hierarchy* H, const saamg_domain* dom, void* stream) {
    return guarded([&] {
        if (!H) throw ApiError{SAAMG_INVALID_ARG, "hierarchy is NULL"};
        HIPCHECK(hipSetDevice(H->device));
        MemScope ms(H->mem, (hipStream_t)stream);
        refresh_impl(H, dom, (hipStream_t)stream);
        return (int)SAAMG_OK;
    });
}

int saamg_destroy(saamg_hierarchy* H) {
    if (!H) return SAAMG_OK;
    // no queued work uses H any more (solves return complete, states are destroyed first)
    MemScope ms(H->mem, nullptr);
    FineLevel& L = H->l0;
    for (void* p : {(void*)L.unk, (void*)L.irr, (void*)L.base, (void*)L.base_full,
                    (void*)L.tab64, (void*)L.tab32, (void*)L.sigma, (void*)H->Ainv,
                    (void*)H->cidx})
        dfree(p);
    for (auto& C : H->lc) free_coarse(C);
    drop_operator(H);
    if (H->ws) {
        state_release(H->ws);
        delete H->ws;
    }
    delete H;
    return SAAMG_OK;
}

int saamg_hierarchy_info(const saamg_hierarchy* H, saamg_info* info) {
    return guarded([&] {
        if (!H || !info) throw ApiError{SAAMG_INVALID_ARG, "NULL argument"};
        std::memset(info, 0, sizeof(*info));
        info->n_levels = H->n_levels;
        info->variant = H->variant;
        info->precision = H->opt.precision;
        for (int l = 0; l < H->n_levels; ++l) {
            int mx, my, mz;
            level_dims(H, l, &mx, &my, &mz);
            info->dims[l][0] = mx;
            info->dims[l][1] = my;
            info->dims[l][2] = mz;
            info->n_unknowns[l] = l == 0 ? H->l0.n_unknowns : H->lc[l - 1].n_unknowns;
            if (l < (int)H->par.size()) {
                info->lambda_est[l] = H->par[l].lam;
                info->omega[l] = H->par[l].omega;
            }
        }
        info->n_irregular = H->l0.n_irr;
        info->device_bytes = H->bytes;
        info->t_setup_ms = H->t_setup_ms;
        info->t_refresh_ms = H->t_refresh_ms;
        for (int q = 0; q < 6; ++q) info->t_setup_phase_ms[q] = H->t_phase_ms[q];
        info->l0_planes = H->l0.zb;
        info->l0_tile_x = H->l0.tx;
        info->l0_wide = H->l0.wide;
        info->l0_wide_planes[0] = H->l0.wzb[1];
        info->l0_wide_planes[1] = H->l0.wzb[0];
        info->table_rows[0] = H->l0.n_tab;
        for (int l = 1; l < H->n_levels; ++l) {
            info->table_rows[l] = H->lc[l - 1].n_tab;
            info->table_rows_t[l] = H->lc[l - 1].sym ? 0 : H->lc[l - 1].n_tabT;
        }
        return (int)SAAMG_OK;
    });
}

static saamg_state* workspace(saamg_hierarchy* H) {
    if (!H->ws) {
        saamg_state* S = new saamg_state();
        try {
            state_alloc(S, H);
        } catch (...) {
            state_release(S);
            delete S;
            throw;
        }
        H->ws = S;
    }
    return H->ws;
}

int saamg_solve(saamg_hierarchy* H, const double* d_b, const double* d_x0, double* d_x, double tol,
                int max_iter, void* stream, saamg_result* res) {
    return guarded([&] {
        if (!H || !d_b || !d_x) throw ApiError{SAAMG_INVALID_ARG, "NULL argument"};
        if (!(tol > 0) || max_iter < 0) throw ApiError{SAAMG_INVALID_ARG, "tol > 0, max_iter >= 0"};
        HIPCHECK(hipSetDevice(H->device));
        auto t0 = std::chrono::steady_clock::now();
        MemScope ms(H->mem, (hipStream_t)stream);
        saamg_state& S = *workspace(H);
        S.s = (hipStream_t)stream;
        S.tol = tol;
        S.max_iter = max_iter;
        state_start(&S, d_b, d_x0);
        while (!S.done) {
            state_enqueue(&S);
            state_complete(&S);
        }
        cg_unscale(cg_op(H), S.x, d_x, S.s);
        HIPCHECK(hipStreamSynchronize(S.s));
        S.s = nullptr;  // the caller's stream is not kept beyond the call
        S.t_ms = ms_since(t0);
        state_fill_result(&S, res);
        return S.status;
    });
}

int saamg_footprint_bytes(int nx, int ny, int nz, int variant, int precision, int64_t* hier_bytes,
                          int64_t* state_bytes) {
    return guarded([&] {
        if (nx < 3 || ny < 3 || nz < 3) throw ApiError{SAAMG_INVALID_ARG, "box must be at least 3^3"};
        const double nbox = (double)nx * ny * nz;
        const bool mixed = precision == SAAMG_MIXED;
        const int na = variant == SAAMG_VARIANT_QUAD ? 27 : 14;
        double h = 8.0 * nbox + 20.0 * nbox / 64 + 0.2 * nbox * 12 * 16;  // sigma, masks, table
        double st = 48.0 * nbox + (mixed ? 4 : 8) * nbox;
        if (l0_wide_default(nx)) {  // the ring of directions in place of the fp64 direction
            const int pw = mixed ? 4 : 8;
            st += (double)(pw * cg_ring_len((long)nbox, pw) - 8) * nbox;
        }
        double w = mixed ? 4 : 8;
        st += 3 * w * nbox + w * nbox / 3;  // level-0 V-cycle vectors and restriction sums
        double m = nbox;
        for (int l = 1; l < 10 && m > 27; ++l) {
            m = (std::ceil(std::cbrt(m) / 3.0) + 2) * (std::ceil(std::cbrt(m) / 3.0) + 2) *
                (std::ceil(std::cbrt(m) / 3.0) + 2);
            // full fp64 arrays and 1/diag, slots, fp32 1/diag, table (at most every row)
            h += ((na + 1) * 8 + (na == 27 ? 8 : 4) + (mixed ? 4 : 0) +
                  (na == 27 ? 2 : 1) * kLcRow * (mixed ? 12 : 8)) * m;
            st += 4 * w * m;
        }
        h += 8.0 * 1000 * 1000;
        if (hier_bytes) *hier_bytes = (int64_t)h;
        if (state_bytes) *state_bytes = (int64_t)st;
        return (int)SAAMG_OK;
    });
}

int saamg_state_create(saamg_hierarchy* H, const double* d_b, const double* d_x0, double tol,
                       int max_iter, void* stream, saamg_state** out) {
    saamg_state* S = nullptr;
    int rc = guarded([&] {
        if (!H || !d_b || !out) throw ApiError{SAAMG_INVALID_ARG, "NULL argument"};
        if (!(tol > 0) || max_iter < 0) throw ApiError{SAAMG_INVALID_ARG, "tol > 0, max_iter >= 0"};
        HIPCHECK(hipSetDevice(H->device));
        MemScope ms(H->mem, (hipStream_t)stream);
        S = new saamg_state();
        S->s = (hipStream_t)stream;
        S->tol = tol;
        S->max_iter = max_iter;
        state_alloc(S, H);
        state_start(S, d_b, d_x0);
        *out = S;
        H->live_states += 1;
        return (int)SAAMG_OK;
    });
    if (rc != SAAMG_OK && S) {
        MemScope ms(H->mem, S->s);
        (void)hipStreamSynchronize(S->s);
        state_release(S);
        delete S;
        if (out) *out = nullptr;
    }
    return rc;
}

int saamg_batch_step(saamg_state* const* states, int n, int* n_done_out) {
    return guarded([&] {
        if (n < 0 || (n > 0 && !states)) throw ApiError{SAAMG_INVALID_ARG, "bad state list"};
        for (int i = 0; i < n; ++i)
            if (!states[i]) throw ApiError{SAAMG_INVALID_ARG, "NULL state"};
        // queue every unfinished state's step on its own stream (a step that
        // saamg_batch_advance queued is already on its way), then collect
        std::vector<saamg_state*> live;
        for (int i = 0; i < n; ++i)
            if (!states[i]->done) {
                auto t0 = std::chrono::steady_clock::now();
                if (!states[i]->inflight) state_enqueue(states[i]);
                states[i]->t_ms += ms_since(t0);
                live.push_back(states[i]);
            }
        for (saamg_state* S : live) {
            auto t0 = std::chrono::steady_clock::now();
            state_complete(S);
            S->t_ms += ms_since(t0);
        }
        int nd = 0;
        for (int i = 0; i < n; ++i) nd += states[i]->done;
        if (n_done_out) *n_done_out = nd;
        return (int)SAAMG_OK;
    });
}

int saamg_batch_advance(saamg_state* const* states, int n, int* n_done_out, int* n_stepped_out) {
    return guarded([&] {
        if (n < 0 || (n > 0 && !states)) throw ApiError{SAAMG_INVALID_ARG, "bad state list"};
        for (int i = 0; i < n; ++i)
            if (!states[i]) throw ApiError{SAAMG_INVALID_ARG, "NULL state"};
        int stepped = 0;
        for (int i = 0; i < n; ++i) {
            saamg_state* S = states[i];
            if (S->done) continue;
            auto t0 = std::chrono::steady_clock::now();
            if (S->inflight) {
                const hipError_t e = hipEventQuery(S->ev);
                if (e == hipErrorNotReady) continue;
                HIPCHECK(e);
                state_complete(S);  // the event has fired: no wait
                stepped += 1;
            }
            if (!S->done) state_enqueue(S);
            S->t_ms += ms_since(t0);
        }
        int nd = 0;
        for (int i = 0; i < n; ++i) nd += states[i]->done;
        if (n_done_out) *n_done_out = nd;
        if (n_stepped_out) *n_stepped_out = stepped;
        return (int)SAAMG_OK;
    });
}

int saamg_state_query(const saamg_state* S, int* done, saamg_result* res) {
    return guarded([&] {
        if (!S) throw ApiError{SAAMG_INVALID_ARG, "NULL state"};
        if (done) *done = S->done;
        state_fill_result(S, res);
        return (int)SAAMG_OK;
    });
}

int saamg_state_finish(saamg_state* S, double* d_x) {
    return guarded([&] {
        if (!S || !d_x) throw ApiError{SAAMG_INVALID_ARG, "NULL argument"};
        HIPCHECK(hipSetDevice(S->H->device));
        if (!S->done) flush_x(S);  // an unfinished state's iterate, with its last step
        cg_unscale(cg_op(S->H), S->x, d_x, S->s);
        HIPCHECK(hipStreamSynchronize(S->s));
        return (int)SAAMG_OK;
    });
}

int saamg_state_destroy(saamg_state* S) {
    if (!S) return SAAMG_OK;
    (void)hipStreamSynchronize(S->s);
    if (S->H) S->H->live_states -= 1;
    MemScope ms(S->H ? S->H->mem : MemCtx{}, S->s);
    state_release(S);
    delete S;
    return SAAMG_OK;
}

int saamg_level_apply(saamg_hierarchy* H, int level, int op, int precision, const double* h_in,
                      double* h_out) {
    return guarded([&] {
        if (!H || !h_in || !h_out) throw ApiError{SAAMG_INVALID_ARG, "NULL argument"};
        if (level < 0 || level >= H->n_levels) throw ApiError{SAAMG_INVALID_ARG, "bad level"};
        if (op < SAAMG_OP_APPLY || op > SAAMG_OP_PROLONG) throw ApiError{SAAMG_INVALID_ARG, "bad op"};
        if (op >= SAAMG_OP_PRESMOOTH && level >= H->n_levels - 1)
            throw ApiError{SAAMG_INVALID_ARG, "no smoother or transfer on the coarsest level"};
        if (precision == SAAMG_MIXED && H->opt.precision != SAAMG_MIXED)
            throw ApiError{SAAMG_INVALID_ARG, "fp32 data exist only for a MIXED hierarchy"};
        HIPCHECK(hipSetDevice(H->device));
        MemScope ms(H->mem, nullptr);
        if (precision == SAAMG_MIXED)
            level_apply_impl<float>(H, level, op, h_in, h_out);
        else
            level_apply_impl<double>(H, level, op, h_in, h_out);
        return (int)SAAMG_OK;
    });
}

int saamg_level_coefficients(saamg_hierarchy* H, int level, double* h_out) {
    return guarded([&] {
        if (!H || !h_out) throw ApiError{SAAMG_INVALID_ARG, "NULL argument"};
        if (level < 0 || level >= H->n_levels) throw ApiError{SAAMG_INVALID_ARG, "bad level"};
        HIPCHECK(hipSetDevice(H->device));
        MemScope ms(H->mem, nullptr);
        int mx, my, mz;
        level_dims(H, level, &mx, &my, &mz);
        const long nlog = (long)mx * my * mz;
        if (level == 0) {
            double* d = (double*)dmalloc(8L * 27 * H->l0.nbox);
            l0_export_coef(H->l0, d, nullptr);
            HIPCHECK(hipMemcpy(h_out, d, 8L * 27 * nlog, hipMemcpyDeviceToHost));
            dfree(d);
            return (int)SAAMG_OK;
        }
        const CoarseLevel& C = H->lc[level - 1];
        std::vector<std::vector<double>> a(27);
        for (int k = 0; k < 27; ++k) {
            if (!C.coef64[k]) continue;
            a[k].resize(C.nstore);
            HIPCHECK(hipMemcpy(a[k].data(), C.coef64[k], 8 * C.nstore, hipMemcpyDeviceToHost));
        }
        for (int k = 0; k < 27; ++k) {
            const int dx = k % 3 - 1, dy = (k / 3) % 3 - 1, dz = k / 9 - 1;
            const long off = dx + (long)C.sx * dy + C.sxy * dz;
            for (int z = 0; z < mz; ++z)
                for (int y = 0; y < my; ++y)
                    for (int x = 0; x < mx; ++x) {
                        const long i = storage_index(H, level, x, y, z);
                        double v = (C.sym && k < 13) ? a[26 - k][i + off] : a[k][i];
                        h_out[k * nlog + x + (long)mx * (y + (long)my * z)] = v;
                    }
        }
        return (int)SAAMG_OK;
    });
}

int saamg_precond_apply(saamg_hierarchy* H, const double* d_r, double* d_z, void* stream) {
    return guarded([&] {
        if (!H || !d_r || !d_z) throw ApiError{SAAMG_INVALID_ARG, "NULL argument"};
        HIPCHECK(hipSetDevice(H->device));
        MemScope ms(H->mem, (hipStream_t)stream);
        saamg_state& S = *workspace(H);
        S.s = (hipStream_t)stream;
        // the residual buffer must stay zero off the unknowns: copy via the scaled mask
        cg_mask_copy(H->l0, d_r, S.r, S.r32, S.s);
        precond(&S, false);
        if (S.mixed)
            f2d_copy((const float*)S.z, d_z, H->l0.nbox, S.s);
        else
            HIPCHECK(hipMemcpyAsync(d_z, S.z, 8 * H->l0.nbox, hipMemcpyDeviceToDevice, S.s));
        HIPCHECK(hipStreamSynchronize(S.s));
        S.s = nullptr;
        return (int)SAAMG_OK;
    });
}

int saamg_operator_apply(saamg_hierarchy* H, const double* d_x, double* d_y, void* stream) {
    return guarded([&] {
        if (!H || !d_x || !d_y) throw ApiError{SAAMG_INVALID_ARG, "NULL argument"};
        if ((reinterpret_cast<uintptr_t>(d_x) | reinterpret_cast<uintptr_t>(d_y)) & 15u)
            throw ApiError{SAAMG_INVALID_ARG, "d_x and d_y must be 16-byte aligned"};
        HIPCHECK(hipSetDevice(H->device));
        l0_apply<double>(cg_op(H), false, d_x, d_y, (hipStream_t)stream);
        HIPCHECK(hipStreamSynchronize((hipStream_t)stream));
        return (int)SAAMG_OK;
    });
}

int saamg_scaling(saamg_hierarchy* H, double* d_sigma, void* stream) {
    return guarded([&] {
        if (!H || !d_sigma) throw ApiError{SAAMG_INVALID_ARG, "NULL argument"};
        HIPCHECK(hipSetDevice(H->device));
        HIPCHECK(hipMemcpyAsync(d_sigma, cg_op(H).sigma, 8 * H->l0.nbox, hipMemcpyDeviceToDevice,
                                (hipStream_t)stream));
        HIPCHECK(hipStreamSynchronize((hipStream_t)stream));
        return (int)SAAMG_OK;
    });
}

int saamg_coarse_inverse(saamg_hierarchy* H, int32_t* n_out, int64_t* h_rows, double* h_inv) {
    return guarded([&] {
        if (!H || !n_out) throw ApiError{SAAMG_INVALID_ARG, "NULL argument"};
        if (!H->Ainv)
            throw ApiError{SAAMG_INVALID_ARG, "the hierarchy has no explicit coarse inverse"};
        *n_out = H->nL;
        if (!h_rows && !h_inv) return (int)SAAMG_OK;
        HIPCHECK(hipSetDevice(H->device));
        const int nL = H->nL, l = H->n_levels - 1;
        if (h_rows) {
            std::vector<long> cidx(nL);
            HIPCHECK(hipMemcpy(cidx.data(), H->cidx, 8L * nL, hipMemcpyDeviceToHost));
            int mx, my, mz;
            level_dims(H, l, &mx, &my, &mz);
            for (int r = 0; r < nL; ++r) {
                long i = cidx[r];
                if (l > 0) {  // padded storage (x + 1) + sx (y + 1) + sxy (z + 1)
                    const CoarseLevel& C = H->lc[l - 1];
                    const long z = i / C.sxy - 1, y = (i % C.sxy) / C.sx - 1, x = i % C.sx - 1;
                    i = x + (long)mx * (y + (long)my * z);
                }
                h_rows[r] = i;
            }
        }
        if (h_inv) HIPCHECK(hipMemcpy(h_inv, H->Ainv, 8L * nL * nL, hipMemcpyDeviceToHost));
        return (int)SAAMG_OK;
    });
}

}  // extern "C"

// ------------------------------------------------------------------ solve without allocation
//
// The work vectors of saamg_solve_noalloc (the PCG vectors, the V-cycle's vectors on every
// level, the block partials and the scalars) are carved out of one file-scope device
// array.  Each device that runs the library holds its own copy until the process ends; in
// host code `scratch` names only a host-side stand-in, so its device address is taken once
// per device with hipGetSymbolAddress and only that address is used.

namespace saamg {

constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static char* g_scratch_ptr[kMaxDevices] = {};

// Device address of the scratch array on `device`, which must be current.
static char* scratch_base(int device) {
    if (device < 0 || device >= kMaxDevices) throw ApiError{SAAMG_INVALID_ARG, "device index"};
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        HIPCHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw ApiError{SAAMG_HIP_ERROR, "no device address for the scratch array"};
        g_scratch_ptr[device] = (char*)p;
    }
    return g_scratch_ptr[device];
}

// Bump allocation from [base, base + cap), 256-byte aligned; nothing is returned.
struct Bump {
    char* base;
    size_t cap, used;
};
static void* bump_alloc(void* ctx, size_t bytes, void*) {
    Bump* b = (Bump*)ctx;
    const size_t off = (b->used + 255) & ~size_t(255);
    if (off > b->cap || bytes > b->cap - off) return nullptr;
    b->used = off + bytes;
    return b->base + off;
}
static void bump_free(void*, void*, void*) {}

// Bytes the work vectors of one solve on H take in the scratch array: the allocation
// sequence of a solve state, run against placeholder addresses (nothing is allocated,
// filled or launched).
static size_t noalloc_bytes(saamg_hierarchy* H) {
    Bump probe{reinterpret_cast<char*>(uintptr_t(256)), ~size_t(0) >> 1, 0};
    MemCtx m;
    m.alloc = bump_alloc;
    m.free = bump_free;
    m.ctx = &probe;
    m.fill = false;
    MemScope ms(m, nullptr);
    saamg_state S;
    state_alloc(&S, H, false);
    S.hscal = nullptr;
    state_release(&S);
    return probe.used;
}

}  // namespace saamg

extern "C" int saamg_solve_noalloc(saamg_hierarchy* H, const double* d_b, const double* d_x0,
                                   double* d_x, double tol, int max_iter, void* stream,
                                   saamg_result* res) {
    return guarded([&] {
        if (!H || !d_b || !d_x) throw ApiError{SAAMG_INVALID_ARG, "NULL argument"};
        if (!(tol > 0) || max_iter < 0) throw ApiError{SAAMG_INVALID_ARG, "tol > 0, max_iter >= 0"};
        HIPCHECK(hipSetDevice(H->device));
        const size_t need = noalloc_bytes(H);
        if (need > kScratchBytes)
            throw ApiError{SAAMG_INVALID_ARG,
                           "the solve needs " + std::to_string(need) + " bytes of work space; the "
                           "scratch array of saamg_solve_noalloc holds " +
                               std::to_string(kScratchBytes) + " bytes (use saamg_solve)"};
        auto t0 = std::chrono::steady_clock::now();
        Bump bump{scratch_base(H->device), kScratchBytes, 0};
        MemCtx m;
        m.alloc = bump_alloc;
        m.free = bump_free;
        m.ctx = &bump;
        MemScope ms(m, (hipStream_t)stream);
        saamg_state S;
        S.s = (hipStream_t)stream;
        S.tol = tol;
        S.max_iter = max_iter;
        state_alloc(&S, H, false);  // zero-filled by a kernel on the stream
        state_start(&S, d_b, d_x0);
        while (!S.done) {
            state_enqueue(&S);
            state_complete(&S);
        }
        cg_unscale(cg_op(H), S.x, d_x, S.s);
        HIPCHECK(hipStreamSynchronize(S.s));
        S.t_ms = ms_since(t0);
        state_fill_result(&S, res);
        S.hscal = nullptr;
        state_release(&S);  // returns nothing: the vectors stay in the scratch array
        return S.status;
    });
}

// ------------------------------------------------------------------ particle coupling

int saamg_pic_create(const saamg_grid* g, const uint8_t* mask, int64_t max_particles,
                     saamg_pic** out) {
    return guarded([&] {
        if (!g || !out) throw ApiError{SAAMG_INVALID_ARG, "NULL argument"};
        *out = nullptr;
        if (g->z_offset != 0 && g->z_offset != 1)
            throw ApiError{SAAMG_INVALID_ARG, "z_offset must be 0 or 1"};
        const int nzl = g->nz - 2 * g->z_offset;
        if (g->nx < 2 || g->ny < 2 || nzl < 2) throw ApiError{SAAMG_INVALID_ARG, "grid too small"};
        if (!(g->h[0] > 0) || !(g->h[1] > 0) || !(g->h[2] > 0) || g->robin_d < 0.0)
            throw ApiError{SAAMG_INVALID_ARG, "spacings must be positive, robin_d >= 0"};
        if (max_particles < 0 || max_particles > 2000000000L)
            throw ApiError{SAAMG_INVALID_ARG, "max_particles must be in 0..2e9"};
        const long ncell = (long)(g->nx - 1) * (g->ny - 1) * (nzl - 1);
        if (ncell >= 4000000000L) throw ApiError{SAAMG_INVALID_ARG, "too many lattice cells"};
        const long nbox = (long)g->nx * g->ny * g->nz;
        MemScope ms(MemCtx{}, nullptr);
        saamg_pic* P = new saamg_pic();
        try {
            HIPCHECK(hipGetDevice(&P->device));
            P->g = *g;
            P->nxl = g->nx;
            P->nyl = g->ny;
            P->nzl = nzl;
            P->ncell = ncell;
            P->cap = max_particles;
            while ((1L << P->key_bits) <= ncell) ++P->key_bits;
            P->mask = (uint8_t*)dmalloc(nbox);
            if (mask) {
                HIPCHECK(hipMemcpy(P->mask, mask, nbox, hipMemcpyHostToDevice));
            } else {
                HIPCHECK(hipMemset(P->mask, 1, nbox));
            }
            const long c = std::max<long>(max_particles, 1);
            P->key = (uint32_t*)dmalloc(4 * c);
            P->key_s = (uint32_t*)dmalloc(4 * c);
            P->idx = (int32_t*)dmalloc(4 * c);
            P->idx_s = (int32_t*)dmalloc(4 * c);
            P->cstart = (int32_t*)dmalloc(4 * ncell);
            P->cend = (int32_t*)dmalloc(4 * ncell);
            P->tmp_bytes = pic_sort_bytes(c, P->key_bits);
            P->tmp = dmalloc(std::max<size_t>(P->tmp_bytes, 16));
            // the fills and the mask upload ran on the null stream: complete them before
            // any stream of the caller uses the context
            HIPCHECK(hipDeviceSynchronize());
        } catch (...) {
            saamg_pic_destroy(P);
            throw;
        }
        *out = P;
        return (int)SAAMG_OK;
    });
}

int saamg_pic_deposit(saamg_pic* P, const double* d_pos, int64_t n, double q, double* d_rho,
                      void* stream) {
    return guarded([&] {
        if (!P || !d_rho || (n > 0 && !d_pos)) throw ApiError{SAAMG_INVALID_ARG, "NULL argument"};
        if (n < 0 || n > P->cap) throw ApiError{SAAMG_INVALID_ARG, "n exceeds the context's capacity"};
        HIPCHECK(hipSetDevice(P->device));
        pic_deposit(P, d_pos, (long)n, q, d_rho, (hipStream_t)stream);
        return (int)SAAMG_OK;
    });
}

int saamg_pic_gather(saamg_pic* P, const double* d_phi, const double* d_pos, int64_t n,
                     double* d_E, void* stream) {
    return guarded([&] {
        if (!P || !d_phi || (n > 0 && (!d_pos || !d_E)))
            throw ApiError{SAAMG_INVALID_ARG, "NULL argument"};
        if (n < 0) throw ApiError{SAAMG_INVALID_ARG, "negative particle count"};
        HIPCHECK(hipSetDevice(P->device));
        pic_gather(P, d_phi, d_pos, (long)n, d_E, (hipStream_t)stream);
        return (int)SAAMG_OK;
    });
}

int saamg_pic_destroy(saamg_pic* P) {
    return guarded([&] {
        if (!P) return (int)SAAMG_OK;
        MemScope ms(MemCtx{}, nullptr);
        for (void* p : {(void*)P->mask, (void*)P->key, (void*)P->key_s, (void*)P->idx,
                        (void*)P->idx_s, (void*)P->cstart, (void*)P->cend, P->tmp})
            if (p) dfree(p);
        delete P;
        return (int)SAAMG_OK;
    });
}
