// extern "C" entry points of include/mlmc.h: argument validation, workspace
// layout and dispatch to the gfx950 kernels.
#include <atomic>
#include <cmath>
#include <mutex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "eigh_large.hpp"
#include "internal.hpp"

using namespace mlmc;

struct mlmc_lattice_s {
    int device = -1;
    DevLattice dev{};
    void *d_buf = nullptr;
};

// Device scratch of mlmc_batched_eigvalsh_noalloc: the two-stage
// reduction's per-matrix workspace for as many matrices as fit, reused chunk
// after chunk.  Each device holds its own copy from the library's load until
// the process ends.  Host code never passes this name to a kernel; it uses
// the device address that hipGetSymbolAddress gives for the current device.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

thread_local std::string g_last_error;

mlmc_status fail(mlmc_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
mlmc_status fail(mlmc_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

mlmc_status hip_fail(hipError_t err, const char *where) {
    return fail(MLMC_ERR_HIP, "%s: %s (%s)", where, hipGetErrorName(err), hipGetErrorString(err));
}

#define HIP_TRY(expr, where)                          \
    do {                                              \
        hipError_t e_ = (expr);                       \
        if (e_ != hipSuccess) return hip_fail(e_, where); \
    } while (0)

// Opt-in launch timing of a context's level estimates
// (mlmc_context_timer / mlmc_context_timer_read): event pairs created when the
// timer is enabled, recorded on the launch stream around each kernel launch.
// The pointer below is set only while a level estimate of a timed context
// enqueues its work on this thread.
struct LaunchTimer {
    std::vector<hipEvent_t> ev;       // 2 * capacity events, created up front
    std::vector<const char *> names;  // name of record r (pair 2r, 2r + 1)
    size_t used = 0;
    int64_t dropped = 0;  // launches not timed because every pair was in use
    bool detail = false;  // also time the kernels inside multi-kernel launchers

    void release() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        ev.clear();
        names.clear();
        used = 0;
        dropped = 0;
    }
};
thread_local LaunchTimer *t_timer = nullptr;

template <typename F>
hipError_t timed(const char *name, hipStream_t s, F &&launch) {
    LaunchTimer *tm = t_timer;
    if (!tm) return launch();
    if (2 * tm->used + 1 >= tm->ev.size()) {
        ++tm->dropped;
        return launch();
    }
    // The record is taken before the launch, so that launches timed inside
    // it (the kernels of a multi-kernel launcher) take the records after it;
    // it gets its name only once both of its events are recorded.
    const size_t r = tm->used;
    tm->names[r] = nullptr;
    tm->used = r + 1;
    hipError_t err = hipEventRecord(tm->ev[2 * r], s);
    if (err != hipSuccess) return err;
    err = launch();
    const hipError_t e2 = hipEventRecord(tm->ev[2 * r + 1], s);
    if (err == hipSuccess && e2 == hipSuccess) tm->names[r] = name;
    return err != hipSuccess ? err : e2;
}

#define LAUNCH(name, stream, expr) HIP_TRY(timed(name, stream, [&]() { return (expr); }), name)

}  // namespace

hipError_t mlmc::timed_sub(const char *name, hipStream_t s, hipError_t (*launch)(void *), void *arg) {
    if (!t_timer || !t_timer->detail) return launch(arg);
    return timed(name, s, [&]() { return launch(arg); });
}

namespace {

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Sequential carving of one workspace; `base == nullptr` only measures.
struct Carver {
    char *base;
    size_t used = 0;
    template <typename P>
    P *take(size_t bytes) {
        const size_t at = used;
        used += align_up(bytes);
        return base ? reinterpret_cast<P *>(base + at) : nullptr;
    }
};

bool valid_lattice(mlmc_lattice lat) { return lat != nullptr && lat->d_buf != nullptr; }

int small_cap(mlmc_precision prec) { return prec == MLMC_PREC_FP64 ? kSmallMaxF64 : kSmallMaxF32; }
int large_cap(mlmc_precision prec) { return prec == MLMC_PREC_FP64 ? kLargeMaxF64 : kLargeMaxF32; }
size_t cplx_bytes(mlmc_precision prec) { return prec == MLMC_PREC_FP64 ? 16 : 8; }

// Buffer sets of a pipelined level estimate: chunks take the sets in turn
// (continuing across calls with one layout), so that the caller's stream can
// start chunk c + 2 while chunk c is still being chased and bisected
// (graphene N = 16, FP64: 22.83k eigensolves/s against 22.73k with two sets;
// one more set of matrices, 8.6 GB there).
constexpr int kLevelSets = 3;

// Buffers of the device-memory eigen path for `units` matrices of side bound ld.
struct EigBuffers {
    void *H = nullptr;
    void *S = nullptr;  // overlap matrices (non-orthogonal basis only)
    double *d = nullptr, *e = nullptr;
    // Further sets 1 .. kLevelSets - 1 for pipelined level estimates (set 0
    // is H, d, e): tridiagonal matrices, and on the two-stage path the
    // matrices themselves (a chunk's chase runs beside the next chunk's stage 1).
    void *Hq[kLevelSets] = {};
    double *dq[kLevelSets] = {}, *eq[kLevelSets] = {};
    void *partial = nullptr;
    int64_t stride = 0;  // complex elements per matrix in `partial` (0: the two-stage layout's size)

    // The view whose H (when it has sets), d, e are set q.
    EigBuffers set(int q) const {
        EigBuffers v = *this;
        if (q > 0) {
            if (Hq[q]) v.H = Hq[q];
            v.d = dq[q];
            v.e = eq[q];
        }
        return v;
    }
};

void carve_tridiagonal(Carver &cv, int64_t ld, int64_t units, int sets, EigBuffers &b) {
    b.d = cv.take<double>(sizeof(double) * (size_t)ld * (size_t)units);
    b.e = cv.take<double>(sizeof(double) * (size_t)ld * (size_t)units);
    for (int q = 1; q < sets; ++q) {
        b.dq[q] = cv.take<double>(sizeof(double) * (size_t)ld * (size_t)units);
        b.eq[q] = cv.take<double>(sizeof(double) * (size_t)ld * (size_t)units);
    }
}

void carve_large(Carver &cv, mlmc_precision prec, int64_t ld, int64_t units, bool with_H, EigBuffers &b,
                 int sets = 1) {
    if (with_H) b.H = cv.take<void>(cplx_bytes(prec) * (size_t)ld * (size_t)ld * (size_t)units);
    for (int q = 1; with_H && q < sets; ++q)
        b.Hq[q] = cv.take<void>(cplx_bytes(prec) * (size_t)ld * (size_t)ld * (size_t)units);
    carve_tridiagonal(cv, ld, units, sets, b);
    const size_t pe = prec == MLMC_PREC_FP64 ? tridiag_twostage_work_elems<double>(ld)
                                             : tridiag_twostage_work_elems<float>(ld);
    b.partial = cv.take<void>(cplx_bytes(prec) * pe * (size_t)units);
}

// Buffers of the generalised path (any ld <= kGenMax): H and S when asked for,
// d, e, and the per-matrix workspace of the Cholesky / two-sided reduction,
// which the two-stage reduction reuses afterwards.
void carve_generalized(Carver &cv, mlmc_precision prec, int64_t ld, int64_t units, bool with_HS, EigBuffers &b,
                       int sets = 1) {
    if (with_HS) {
        b.H = cv.take<void>(cplx_bytes(prec) * (size_t)ld * (size_t)ld * (size_t)units);
        b.S = cv.take<void>(cplx_bytes(prec) * (size_t)ld * (size_t)ld * (size_t)units);
    }
    for (int q = 1; with_HS && q < sets; ++q)  // C = L^-1 H L^-H stays in H, which the chase reads
        b.Hq[q] = cv.take<void>(cplx_bytes(prec) * (size_t)ld * (size_t)ld * (size_t)units);
    carve_tridiagonal(cv, ld, units, sets, b);
    const size_t pe = prec == MLMC_PREC_FP64 ? generalized_work_elems<double>(ld) : generalized_work_elems<float>(ld);
    b.partial = cv.take<void>(cplx_bytes(prec) * pe * (size_t)units);
    b.stride = (int64_t)pe;  // the two-stage kernels use the same per-matrix spacing as the Cholesky ones
}

// Eigenvalues of `units` matrices already in b.H (ld > small cap).  With
// defer_bisect the tridiagonal matrices are left in b.d, b.e and the caller
// runs the bisection (run_bisect) itself.
mlmc_status run_bisect(const int32_t *n, int64_t ld, int64_t units, double *w, int64_t ldw, const EigBuffers &b,
                       hipStream_t s, int64_t max_blocks = 0) {
    LAUNCH("bisect", s, launch_bisect(b.d, b.e, ld, n, units, ld, w, ldw, s, max_blocks));
    return MLMC_OK;
}

// Band -> tridiagonal (b.d, b.e) of matrices that stage 1 left in H, on at
// most max_blocks workgroups (0: one per matrix).
mlmc_status run_chase(mlmc_precision prec, const void *H, int64_t ld, const int32_t *n, int64_t units,
                      const EigBuffers &b, hipStream_t s, int64_t max_blocks = 0, const int64_t *offs = nullptr) {
    if (prec == MLMC_PREC_FP64)
        LAUNCH("chase", s, launch_band_chase<double>(static_cast<const cpx<double> *>(H), ld, n, units, b.d, b.e, ld,
                                                     static_cast<cpx<double> *>(b.partial), s, max_blocks, b.stride,
                                                     offs));
    else
        LAUNCH("chase", s, launch_band_chase<float>(static_cast<const cpx<float> *>(H), ld, n, units, b.d, b.e, ld,
                                                    static_cast<cpx<float> *>(b.partial), s, max_blocks, b.stride,
                                                    offs));
    return MLMC_OK;
}

// With defer_chase only stage 1 runs here (the caller runs run_chase and
// run_bisect, possibly on other streams).  offs: element offset of each
// matrix in H (NULL: u ld^2).
mlmc_status run_large(mlmc_precision prec, void *H, int64_t ld, const int32_t *n, int64_t units, double *w, int64_t ldw,
                      const EigBuffers &b, hipStream_t s, bool defer_bisect = false, bool defer_chase = false,
                      const int64_t *offs = nullptr, int upd_rows = 32) {
    if (prec == MLMC_PREC_FP64)
        LAUNCH("band_reduce", s, launch_band_reduce<double>(static_cast<cpx<double> *>(H), ld, n, units,
                                                            static_cast<cpx<double> *>(b.partial), s, b.stride, offs,
                                                            upd_rows));
    else
        LAUNCH("band_reduce", s, launch_band_reduce<float>(static_cast<cpx<float> *>(H), ld, n, units,
                                                           static_cast<cpx<float> *>(b.partial), s, b.stride, offs,
                                                           upd_rows));
    if (defer_chase) return MLMC_OK;
    const mlmc_status st = run_chase(prec, H, ld, n, units, b, s, 0, offs);
    if (st != MLMC_OK || defer_bisect) return st;
    return run_bisect(n, ld, units, w, ldw, b, s);
}

// Layout of mlmc_level_estimate's workspace for a chunk of `mc` samples.  The
// matrices (two-stage path), matrix sizes, tridiagonal matrices and
// eigenvalues come in kLevelSets sets, used by chunks in turn, so that one
// chunk's chase, bisection and IDoS overlap the reduction of the next ones.
struct LevelLayout {
    // k-points and weights per set: a chunk rewrites its set's copy only after
    // the back stream has released the set, so a following call with the same
    // layout never writes a k-grid that an earlier chunk's IDoS still reads.
    double *kf[kLevelSets] = {}, *kwf[kLevelSets] = {}, *kc[kLevelSets] = {}, *kwc[kLevelSets] = {};
    uint8_t *mask = nullptr, *quarters = nullptr;
    int32_t *nf[kLevelSets] = {}, *nc[kLevelSets] = {};
    double *wf[kLevelSets] = {}, *wc[kLevelSets] = {};
    double *If = nullptr, *Ic = nullptr;
    EigBuffers bf, bc;
    int sets = kLevelSets;  // buffer sets in use (1: a single pass)
    size_t bytes = 0;
};

static bool valid_kgrid_kind(int kind) {
    return kind == MLMC_KGRID_MP || kind == MLMC_KGRID_GAMMA || kind == MLMC_KGRID_RHOMBI;
}

LevelLayout level_layout(const mlmc_lattice_s *lat, int N, bool coupled, int Kf, int Kc, int kind, int64_t mc,
                         mlmc_precision prec, int n_eps, char *base, int sets = kLevelSets) {
    LevelLayout L;
    L.sets = sets;
    Carver cv{base};
    const int G = lat->dev.n_groups, no = lat->dev.n_orb;
    const int64_t nkf = kgrid_count(kind, Kf), nkc = kgrid_count(kind, Kc);
    const int64_t ldf = (int64_t)no * N * N;
    for (int q = 0; q < sets; ++q) {
        L.kf[q] = cv.take<double>(sizeof(double) * 2 * nkf);
        L.kwf[q] = cv.take<double>(sizeof(double) * nkf);
    }
    L.mask = cv.take<uint8_t>((size_t)mc * N * N * G);
    for (int q = 0; q < sets; ++q) {
        L.nf[q] = cv.take<int32_t>(sizeof(int32_t) * (size_t)(mc * nkf));
        L.wf[q] = cv.take<double>(sizeof(double) * (size_t)(mc * nkf * ldf));
    }
    L.If = cv.take<double>(sizeof(double) * (size_t)mc * n_eps);
    const bool gen = lat->dev.n_ovl > 0;
    if (gen) carve_generalized(cv, prec, ldf, mc * nkf, true, L.bf, sets);
    else if (ldf > small_cap(prec)) carve_large(cv, prec, ldf, mc * nkf, true, L.bf, sets);
    if (coupled) {
        const int h = N / 2;
        const int64_t ldc = (int64_t)no * h * h;
        for (int q = 0; q < sets; ++q) {
            L.kc[q] = cv.take<double>(sizeof(double) * 2 * nkc);
            L.kwc[q] = cv.take<double>(sizeof(double) * nkc);
        }
        L.quarters = cv.take<uint8_t>((size_t)mc * 4 * h * h * G);
        for (int q = 0; q < sets; ++q) {
            L.nc[q] = cv.take<int32_t>(sizeof(int32_t) * (size_t)(mc * 4 * nkc));
            L.wc[q] = cv.take<double>(sizeof(double) * (size_t)(mc * 4 * nkc * ldc));
        }
        L.Ic = cv.take<double>(sizeof(double) * (size_t)mc * 4 * n_eps);
        if (gen) carve_generalized(cv, prec, ldc, mc * 4 * nkc, true, L.bc, sets);
        else if (ldc > small_cap(prec)) carve_large(cv, prec, ldc, mc * 4 * nkc, true, L.bc, sets);
    }
    L.bytes = cv.used;
    return L;
}

// Pencils (H, S) already in b.H, b.S -> eigenvalues (reduction to C = L^{-1}
// H L^{-H}, then the standard path on C).
mlmc_status run_generalized(mlmc_precision prec, void *H, void *S, int64_t ld, const int32_t *n, int64_t units,
                            double *w, int64_t ldw, const EigBuffers &b, hipStream_t s, bool *bisect_pending = nullptr,
                            bool *chase_pending = nullptr, int upd_rows = 32) {
    if (prec == MLMC_PREC_FP64)
        LAUNCH("overlap_reduce", s, launch_cholesky_reduce<double>(static_cast<cpx<double> *>(H), static_cast<cpx<double> *>(S), ld, n, units,
                                                            static_cast<cpx<double> *>(b.partial), s));
    else
        LAUNCH("overlap_reduce", s, launch_cholesky_reduce<float>(static_cast<cpx<float> *>(H), static_cast<cpx<float> *>(S), ld, n, units,
                                                           static_cast<cpx<float> *>(b.partial), s));
    if (ld <= small_cap(prec)) {
        if (prec == MLMC_PREC_FP64)
            LAUNCH("small_fused", s, launch_small_from_matrix<double>(static_cast<const cpx<double> *>(H), ld, n, units, w, ldw, s));
        else
            LAUNCH("small_fused", s, launch_small_from_matrix<float>(static_cast<const cpx<float> *>(H), ld, n, units, w, ldw, s));
        return MLMC_OK;
    }
    if (bisect_pending) *bisect_pending = true;
    if (bisect_pending && chase_pending) *chase_pending = true;
    return run_large(prec, H, ld, n, units, w, ldw, b, s, bisect_pending != nullptr,
                     bisect_pending != nullptr && chase_pending != nullptr, nullptr, upd_rows);
}

// Eigenvalues of every (outcome, k) unit of `ns` outcomes of side N.  With
// bisect_pending, a path that ends in a bisection stops before it and says so
// (the caller then calls run_bisect on the same buffers); with chase_pending
// as well, the two-stage path stops after stage 1 (the caller then calls
// run_chase first).
mlmc_status outcome_spectra(const mlmc_lattice_s *lat, int N, const uint8_t *mask, int64_t ns, const double *kred,
                            int nk, mlmc_precision prec, double *w, int32_t *n_out, const EigBuffers &b,
                            hipStream_t s, bool *bisect_pending = nullptr, bool *chase_pending = nullptr,
                            int upd_rows = 32) {
    const int64_t ld = (int64_t)lat->dev.n_orb * N * N;
    const int64_t units = ns * nk;
    if (bisect_pending) *bisect_pending = false;
    if (chase_pending) *chase_pending = false;
    // The eigensolvers read lower triangles only, so only those are assembled.
    if (lat->dev.n_ovl > 0) {  // non-orthogonal basis: assemble H and S, generalised path
        if (prec == MLMC_PREC_FP64) {
            LAUNCH("assemble", s, launch_assemble<double>(lat->dev, N, mask, ns, kred, nk, static_cast<cpx<double> *>(b.H), ld, n_out, s, false, true));
            LAUNCH("assemble", s, launch_assemble<double>(lat->dev, N, mask, ns, kred, nk, static_cast<cpx<double> *>(b.S), ld, n_out, s, true, true));
        } else {
            LAUNCH("assemble", s, launch_assemble<float>(lat->dev, N, mask, ns, kred, nk, static_cast<cpx<float> *>(b.H), ld, n_out, s, false, true));
            LAUNCH("assemble", s, launch_assemble<float>(lat->dev, N, mask, ns, kred, nk, static_cast<cpx<float> *>(b.S), ld, n_out, s, true, true));
        }
        return run_generalized(prec, b.H, b.S, ld, n_out, units, w, ld, b, s, bisect_pending, chase_pending, upd_rows);
    }
    if (ld <= small_cap(prec)) {
        if (prec == MLMC_PREC_FP64)
            LAUNCH("small_fused", s, launch_small_from_lattice<double>(lat->dev, N, mask, ns, kred, nk, w, ld, n_out, s));
        else
            LAUNCH("small_fused", s, launch_small_from_lattice<float>(lat->dev, N, mask, ns, kred, nk, w, ld, n_out, s));
        return MLMC_OK;
    }
    if (prec == MLMC_PREC_FP64)
        LAUNCH("assemble", s, launch_assemble<double>(lat->dev, N, mask, ns, kred, nk, static_cast<cpx<double> *>(b.H), ld, n_out, s, false, true));
    else
        LAUNCH("assemble", s, launch_assemble<float>(lat->dev, N, mask, ns, kred, nk, static_cast<cpx<float> *>(b.H), ld, n_out, s, false, true));
    if (bisect_pending) *bisect_pending = true;
    if (bisect_pending && chase_pending) *chase_pending = true;
    return run_large(prec, b.H, ld, n_out, units, w, ld, b, s, bisect_pending != nullptr,
                     bisect_pending != nullptr && chase_pending != nullptr, nullptr, upd_rows);
}

// Workgroups (one per CU) of a chase on a context's chase stream: the next
// chunk's stage 1 runs on the quarter of the CUs it leaves free and, with the
// 32-row rank-2k update, beside it on the others (measured on the graphene
// N = 16 workload: FP64 3/4 of the CUs 24.7k eigensolves/s, 5/8 22.9k, 7/8
// 24.1k, all 21.9k; mixed 40.3k, 37.6k, 38.8k, 30.1k).
int64_t chase_cus(int cus) {
    const int64_t v = (int64_t)cus * 3 / 4;
    return v > 0 ? v : 1;
}

// Workspace layout of a level estimate: calls with equal keys use the
// workspace's buffer sets in the same places.
struct LayoutKey {
    const void *work = nullptr;
    int64_t mc = 0, nkf = 0, nkc = 0;
    int n_orb = 0, n_groups = 0, N = 0, n_eps = 0, prec = 0, sets = 0;
    bool cpl = false, gen = false;
    bool operator==(const LayoutKey &o) const {
        return work == o.work && mc == o.mc && nkf == o.nkf && nkc == o.nkc && n_orb == o.n_orb &&
               n_groups == o.n_groups && N == o.N && n_eps == o.n_eps && prec == o.prec && sets == o.sets &&
               cpl == o.cpl && gen == o.gen;
    }
};

}  // namespace

// A pipeline context (mlmc_context_create): the two streams of a pipelined
// level estimate besides the caller's (back: bisection, IDoS, level sums;
// chase), the events that order them, the rotation state of consecutive
// calls, and an optional launch timer.  Everything a level estimate keeps
// between calls lives here, so calls on different contexts share nothing.
struct mlmc_context_s {
    int device = -1;
    hipStream_t s = nullptr;      // back stream
    hipStream_t sc = nullptr;     // chase stream
    hipStream_t front[2] = {};    // two caller streams the context offers (mlmc_context_stream)
    int64_t bisect_blocks = 0;    // workgroups of a bisection on the back stream: one per CU
    int64_t chase_blocks = 0;     // workgroups of a chase on the chase stream
    hipEvent_t begin = nullptr;   // caller's stream -> back stream
    hipEvent_t ready = nullptr;   // front (caller's stream) -> chase and back: a chunk's front part is complete
    hipEvent_t chased = nullptr;  // chase -> back: a chunk's tridiagonals are complete
    hipEvent_t freed[kLevelSets] = {};  // back -> front: set q of the matrices / sizes / tridiagonals /
                                        // eigenvalues is free
    hipEvent_t end = nullptr;     // back -> caller's stream
    // The previous level estimate's workspace layout and the set its next
    // chunk would use.  A call with the same layout continues the rotation:
    // each of its chunks waits only for the release of its own set (and its
    // first for the previous call's front part), so it may start while the
    // previous call's last chunks are still chased and bisected.
    LayoutKey last;
    int next_set = 0;
    hipStream_t last_stream = nullptr;  // the previous call's stream
    int upd_rows = 32;                  // rows of the stage-1 update tiles (32 or 64)
    std::mutex mu;                      // held while a call enqueues its work on this context
    LaunchTimer timer;

    // Destroys every HIP object the context holds (after its streams are idle).
    hipError_t release() {
        hipError_t err = hipSuccess;
        auto keep = [&](hipError_t e) {
            if (err == hipSuccess && e != hipSuccess) err = e;
        };
        if (sc) keep(hipStreamSynchronize(sc));
        if (s) keep(hipStreamSynchronize(s));
        timer.release();
        hipEvent_t *evs[4 + kLevelSets] = {&begin, &ready, &chased, &end};
        for (int q = 0; q < kLevelSets; ++q) evs[4 + q] = &freed[q];
        for (hipEvent_t *ev : evs) {
            if (*ev) keep(hipEventDestroy(*ev));
            *ev = nullptr;
        }
        if (sc) keep(hipStreamDestroy(sc));
        if (s) keep(hipStreamDestroy(s));
        sc = s = nullptr;
        for (hipStream_t &f : front) {
            if (f) {
                keep(hipStreamSynchronize(f));
                keep(hipStreamDestroy(f));
            }
            f = nullptr;
        }
        return err;
    }
};

namespace {

mlmc_status convert_hops(const mlmc_lattice_desc *desc, const mlmc_hop *rows, int count, const char *what,
                         std::vector<int4> &hi, std::vector<double4> &hf) {
    hi.resize(count);
    hf.resize(count);
    for (int h = 0; h < count; ++h) {
        const mlmc_hop &r = rows[h];
        if (r.from_orb < 0 || r.from_orb >= desc->n_orb || r.to_orb < 0 || r.to_orb >= desc->n_orb)
            return fail(MLMC_ERR_INVALID_ARG, "%s %d: orbital out of range", what, h);
        if (!std::isfinite(r.re) || !std::isfinite(r.im))
            return fail(MLMC_ERR_INVALID_ARG, "%s %d: non-finite amplitude", what, h);
        const bool onsite = r.R[0] == 0 && r.R[1] == 0 && r.from_orb == r.to_orb;
        if (onsite && r.im != 0.0) return fail(MLMC_ERR_INVALID_ARG, "%s %d: on-site entry must be real", what, h);
        hi[h] = make_int4(r.R[0], r.R[1], r.from_orb, r.to_orb);
        const double d1 = r.R[0] + desc->orb_frac[2 * r.to_orb] - desc->orb_frac[2 * r.from_orb];
        const double d2 = r.R[1] + desc->orb_frac[2 * r.to_orb + 1] - desc->orb_frac[2 * r.from_orb + 1];
        hf[h] = make_double4(r.re, r.im, d1, d2);
    }
    return MLMC_OK;
}

}  // namespace

extern "C" {

const char *mlmc_status_string(int status) {
    switch (status) {
        case MLMC_OK: return "MLMC_OK";
        case MLMC_ERR_INVALID_ARG: return "MLMC_ERR_INVALID_ARG";
        case MLMC_ERR_UNSUPPORTED: return "MLMC_ERR_UNSUPPORTED";
        case MLMC_ERR_WORKSPACE: return "MLMC_ERR_WORKSPACE";
        case MLMC_ERR_HIP: return "MLMC_ERR_HIP";
        default: return "MLMC_ERR_UNKNOWN";
    }
}

const char *mlmc_last_error(void) { return g_last_error.c_str(); }

mlmc_status mlmc_lattice_create(const mlmc_lattice_desc *desc, mlmc_lattice *out) {
    if (!desc || !out) return fail(MLMC_ERR_INVALID_ARG, "lattice_create: NULL argument");
    *out = nullptr;
    if (desc->n_orb < 1 || desc->n_orb > 64) return fail(MLMC_ERR_INVALID_ARG, "n_orb out of range: %d", desc->n_orb);
    if (desc->n_groups < 1 || desc->n_groups > 16)
        return fail(MLMC_ERR_INVALID_ARG, "n_groups out of range: %d", desc->n_groups);
    if (desc->n_hops < 1 || desc->n_hops > 65536)
        return fail(MLMC_ERR_INVALID_ARG, "n_hops out of range: %d", desc->n_hops);
    if (!(desc->cell_area > 0.0)) return fail(MLMC_ERR_INVALID_ARG, "cell_area must be > 0");
    if (!desc->orb_frac || !desc->orb_group || !desc->group_removable || !desc->hops)
        return fail(MLMC_ERR_INVALID_ARG, "lattice_create: NULL array");
    for (int m = 0; m < desc->n_orb; ++m)
        if (desc->orb_group[m] < 0 || desc->orb_group[m] >= desc->n_groups)
            return fail(MLMC_ERR_INVALID_ARG, "orb_group[%d] out of range", m);
    if (desc->n_overlap < 0 || desc->n_overlap > 65536 || (desc->n_overlap > 0 && !desc->overlap))
        return fail(MLMC_ERR_INVALID_ARG, "n_overlap out of range or NULL overlap table");
    std::vector<int4> hi, oi;
    std::vector<double4> hf, of;
    mlmc_status st = convert_hops(desc, desc->hops, desc->n_hops, "hop", hi, hf);
    if (st != MLMC_OK) return st;
    st = convert_hops(desc, desc->overlap, desc->n_overlap, "overlap", oi, of);
    if (st != MLMC_OK) return st;
    auto *lat = new mlmc_lattice_s();
    HIP_TRY(hipGetDevice(&lat->device), "hipGetDevice");
    const int no = desc->n_overlap;
    const size_t bi = align_up(sizeof(int4) * desc->n_hops), bf = align_up(sizeof(double4) * desc->n_hops);
    const size_t bg = align_up(sizeof(int32_t) * desc->n_orb), br = align_up(desc->n_groups);
    const size_t boi = align_up(sizeof(int4) * no), bof = align_up(sizeof(double4) * no);
    hipError_t err = hipMalloc(&lat->d_buf, bi + bf + bg + br + boi + bof);
    if (err != hipSuccess) {
        delete lat;
        return hip_fail(err, "hipMalloc(lattice)");
    }
    char *p = static_cast<char *>(lat->d_buf);
    char *po = p + bi + bf + bg + br;
    err = hipMemcpy(p, hi.data(), sizeof(int4) * desc->n_hops, hipMemcpyHostToDevice);
    if (err == hipSuccess) err = hipMemcpy(p + bi, hf.data(), sizeof(double4) * desc->n_hops, hipMemcpyHostToDevice);
    if (err == hipSuccess) err = hipMemcpy(p + bi + bf, desc->orb_group, sizeof(int32_t) * desc->n_orb, hipMemcpyHostToDevice);
    if (err == hipSuccess) err = hipMemcpy(p + bi + bf + bg, desc->group_removable, desc->n_groups, hipMemcpyHostToDevice);
    if (err == hipSuccess && no > 0) err = hipMemcpy(po, oi.data(), sizeof(int4) * no, hipMemcpyHostToDevice);
    if (err == hipSuccess && no > 0) err = hipMemcpy(po + boi, of.data(), sizeof(double4) * no, hipMemcpyHostToDevice);
    if (err != hipSuccess) {
        (void)hipFree(lat->d_buf);
        delete lat;
        return hip_fail(err, "hipMemcpy(lattice)");
    }
    lat->dev.hop_i = reinterpret_cast<const int4 *>(p);
    lat->dev.hop_f = reinterpret_cast<const double4 *>(p + bi);
    lat->dev.orb_group = reinterpret_cast<const int32_t *>(p + bi + bf);
    lat->dev.removable = reinterpret_cast<const uint8_t *>(p + bi + bf + bg);
    lat->dev.ovl_i = no > 0 ? reinterpret_cast<const int4 *>(po) : nullptr;
    lat->dev.ovl_f = no > 0 ? reinterpret_cast<const double4 *>(po + boi) : nullptr;
    lat->dev.n_ovl = no;
    lat->dev.n_orb = desc->n_orb;
    lat->dev.n_groups = desc->n_groups;
    lat->dev.n_hops = desc->n_hops;
    lat->dev.lattice_id = desc->lattice_id;
    lat->dev.cell_area = desc->cell_area;
    *out = lat;
    return MLMC_OK;
}

mlmc_status mlmc_lattice_destroy(mlmc_lattice lat) {
    if (!lat) return MLMC_OK;
    hipError_t err = hipSuccess;
    if (lat->d_buf) {
        err = hipDeviceSynchronize();
        const hipError_t e2 = hipFree(lat->d_buf);
        if (err == hipSuccess) err = e2;
    }
    delete lat;
    if (err != hipSuccess) return hip_fail(err, "lattice_destroy");
    return MLMC_OK;
}

mlmc_status mlmc_lattice_max_orbitals(mlmc_lattice lat, int32_t N, int64_t *n_max) {
    if (!valid_lattice(lat) || !n_max || N < 1) return fail(MLMC_ERR_INVALID_ARG, "lattice_max_orbitals: bad argument");
    *n_max = (int64_t)lat->dev.n_orb * N * N;
    return MLMC_OK;
}

mlmc_status mlmc_sample_vacancies(mlmc_lattice lat, int32_t N, double p, uint64_t seed, uint64_t tag,
                                  int64_t first_sample, int64_t n_samples, uint8_t *d_mask, mlmc_stream stream) {
    if (!valid_lattice(lat)) return fail(MLMC_ERR_INVALID_ARG, "sample_vacancies: NULL lattice");
    if (N < 1 || N > 4096) return fail(MLMC_ERR_INVALID_ARG, "sample_vacancies: N = %d", N);
    if (!(p >= 0.0 && p <= 1.0)) return fail(MLMC_ERR_INVALID_ARG, "sample_vacancies: p = %g", p);
    if (n_samples < 0 || first_sample < 0) return fail(MLMC_ERR_INVALID_ARG, "sample_vacancies: negative count");
    if (n_samples > 0 && !d_mask) return fail(MLMC_ERR_INVALID_ARG, "sample_vacancies: NULL mask");
    const uint64_t thr = (uint64_t)std::floor(p * 9007199254740992.0);
    LAUNCH("sample_vacancies", static_cast<hipStream_t>(stream), launch_sample_vacancies(lat->dev, N, thr, seed, tag, first_sample, n_samples, d_mask,
                                    static_cast<hipStream_t>(stream)));
    return MLMC_OK;
}

mlmc_status mlmc_partition_masks(mlmc_lattice lat, int32_t N, const uint8_t *d_mask, int64_t n_samples,
                                 uint8_t *d_quarters, mlmc_stream stream) {
    if (!valid_lattice(lat)) return fail(MLMC_ERR_INVALID_ARG, "partition_masks: NULL lattice");
    if (N < 2 || N % 2 != 0) return fail(MLMC_ERR_INVALID_ARG, "partition_masks: N = %d must be even", N);
    if (n_samples < 0) return fail(MLMC_ERR_INVALID_ARG, "partition_masks: negative count");
    if (n_samples > 0 && (!d_mask || !d_quarters)) return fail(MLMC_ERR_INVALID_ARG, "partition_masks: NULL buffer");
    LAUNCH("partition", static_cast<hipStream_t>(stream), launch_partition(N, lat->dev.n_groups, d_mask, n_samples, d_quarters, static_cast<hipStream_t>(stream)));
    return MLMC_OK;
}

mlmc_status mlmc_kgrid_points(mlmc_kgrid_kind kind, int32_t K, int32_t *n_k) {
    if (!valid_kgrid_kind(kind)) return fail(MLMC_ERR_INVALID_ARG, "kgrid_points: bad kind");
    if (K < 1 || K > 4096) return fail(MLMC_ERR_INVALID_ARG, "kgrid_points: K = %d", K);
    if (!n_k) return fail(MLMC_ERR_INVALID_ARG, "kgrid_points: NULL n_k");
    *n_k = kgrid_count(kind, K);
    return MLMC_OK;
}

mlmc_status mlmc_kgrid(mlmc_kgrid_kind kind, int32_t K, double *d_kred, double *d_kweight, mlmc_stream stream) {
    if (!valid_kgrid_kind(kind)) return fail(MLMC_ERR_INVALID_ARG, "kgrid: bad kind");
    if (K < 1 || K > 4096) return fail(MLMC_ERR_INVALID_ARG, "kgrid: K = %d", K);
    if (!d_kred || !d_kweight) return fail(MLMC_ERR_INVALID_ARG, "kgrid: NULL buffer");
    LAUNCH("kgrid", static_cast<hipStream_t>(stream), launch_kgrid(kind, K, d_kred, d_kweight, static_cast<hipStream_t>(stream)));
    return MLMC_OK;
}

mlmc_status mlmc_build_hamiltonians(mlmc_lattice lat, int32_t N, const uint8_t *d_mask, int64_t n_samples,
                                    const double *d_kred, int32_t n_k, mlmc_dtype dtype, void *d_H, int64_t ld,
                                    int32_t *d_n, mlmc_stream stream) {
    if (!valid_lattice(lat)) return fail(MLMC_ERR_INVALID_ARG, "build_hamiltonians: NULL lattice");
    if (N < 1 || N > 4096 || n_k < 1 || n_samples < 0)
        return fail(MLMC_ERR_INVALID_ARG, "build_hamiltonians: N = %d, n_k = %d", N, n_k);
    if (dtype != MLMC_C128 && dtype != MLMC_C64) return fail(MLMC_ERR_INVALID_ARG, "build_hamiltonians: bad dtype");
    const int64_t nmax = (int64_t)lat->dev.n_orb * N * N;
    if (ld < nmax) return fail(MLMC_ERR_INVALID_ARG, "build_hamiltonians: ld %lld < %lld", (long long)ld, (long long)nmax);
    if (nmax > 16384) return fail(MLMC_ERR_UNSUPPORTED, "build_hamiltonians: %lld orbitals exceed 16384", (long long)nmax);
    if (n_samples > 0 && (!d_mask || !d_kred || !d_H || !d_n))
        return fail(MLMC_ERR_INVALID_ARG, "build_hamiltonians: NULL buffer");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (dtype == MLMC_C128)
        LAUNCH("assemble", s, launch_assemble<double>(lat->dev, N, d_mask, n_samples, d_kred, n_k, static_cast<cpx<double> *>(d_H), ld,
                                        d_n, s));
    else
        LAUNCH("assemble", s, launch_assemble<float>(lat->dev, N, d_mask, n_samples, d_kred, n_k, static_cast<cpx<float> *>(d_H), ld,
                                       d_n, s));
    return MLMC_OK;
}

mlmc_status mlmc_build_overlaps(mlmc_lattice lat, int32_t N, const uint8_t *d_mask, int64_t n_samples,
                                const double *d_kred, int32_t n_k, mlmc_dtype dtype, void *d_S, int64_t ld,
                                int32_t *d_n, mlmc_stream stream) {
    if (!valid_lattice(lat)) return fail(MLMC_ERR_INVALID_ARG, "build_overlaps: NULL lattice");
    if (lat->dev.n_ovl < 1) return fail(MLMC_ERR_INVALID_ARG, "build_overlaps: the lattice has no overlap table");
    if (N < 1 || N > 4096 || n_k < 1 || n_samples < 0)
        return fail(MLMC_ERR_INVALID_ARG, "build_overlaps: N = %d, n_k = %d", N, n_k);
    if (dtype != MLMC_C128 && dtype != MLMC_C64) return fail(MLMC_ERR_INVALID_ARG, "build_overlaps: bad dtype");
    const int64_t nmax = (int64_t)lat->dev.n_orb * N * N;
    if (ld < nmax) return fail(MLMC_ERR_INVALID_ARG, "build_overlaps: ld %lld < %lld", (long long)ld, (long long)nmax);
    if (nmax > 16384) return fail(MLMC_ERR_UNSUPPORTED, "build_overlaps: %lld orbitals exceed 16384", (long long)nmax);
    if (n_samples > 0 && (!d_mask || !d_kred || !d_S || !d_n))
        return fail(MLMC_ERR_INVALID_ARG, "build_overlaps: NULL buffer");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (dtype == MLMC_C128)
        LAUNCH("assemble", s, launch_assemble<double>(lat->dev, N, d_mask, n_samples, d_kred, n_k,
                                                      static_cast<cpx<double> *>(d_S), ld, d_n, s, true));
    else
        LAUNCH("assemble", s, launch_assemble<float>(lat->dev, N, d_mask, n_samples, d_kred, n_k,
                                                     static_cast<cpx<float> *>(d_S), ld, d_n, s, true));
    return MLMC_OK;
}

static mlmc_status check_dtype_prec(mlmc_dtype dtype, mlmc_precision prec) {
    if (dtype == MLMC_C128 && prec == MLMC_PREC_FP64) return MLMC_OK;
    if (dtype == MLMC_C64 && prec == MLMC_PREC_MIXED) return MLMC_OK;
    return fail(MLMC_ERR_UNSUPPORTED, "dtype %d with precision %d is not supported", (int)dtype, (int)prec);
}

static mlmc_status eigvalsh_workspace(mlmc_dtype dtype, mlmc_precision prec, int64_t ld, int64_t batch, size_t *bytes) {
    if (!bytes || ld < 0 || batch < 0) return fail(MLMC_ERR_INVALID_ARG, "eigvalsh_workspace: bad argument");
    const mlmc_status st = check_dtype_prec(dtype, prec);
    if (st != MLMC_OK) return st;
    if (ld > large_cap(prec)) return fail(MLMC_ERR_UNSUPPORTED, "eigvalsh: ld %lld exceeds %d", (long long)ld, large_cap(prec));
    *bytes = 0;
    if (ld > small_cap(prec)) {
        Carver cv{nullptr};
        EigBuffers b;
        carve_large(cv, prec, ld, batch, false, b);
        *bytes = cv.used;
    }
    return MLMC_OK;
}

mlmc_status mlmc_batched_eigvalsh(mlmc_dtype dtype, mlmc_precision prec, void *d_H, int64_t ld,
                                  const int64_t *d_offsets, const int32_t *d_n, int64_t batch, double *d_w, int64_t ldw,
                                  void *d_work, size_t work_bytes, mlmc_stream stream) {
    size_t need = 0;
    const mlmc_status st = eigvalsh_workspace(dtype, prec, ld, batch, &need);
    if (st != MLMC_OK) return st;
    if (ldw < ld) return fail(MLMC_ERR_INVALID_ARG, "batched_eigvalsh: ldw %lld < ld %lld", (long long)ldw, (long long)ld);
    if (batch > 0 && (!d_H || !d_n || !d_w)) return fail(MLMC_ERR_INVALID_ARG, "batched_eigvalsh: NULL buffer");
    if (need > 0 && (!d_work || work_bytes < need))
        return fail(MLMC_ERR_WORKSPACE, "batched_eigvalsh: workspace %zu < %zu bytes", work_bytes, need);
    if (batch == 0 || ld == 0) return MLMC_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (ld <= small_cap(prec)) {
        if (prec == MLMC_PREC_FP64)
            LAUNCH("small_fused", s, launch_small_from_matrix<double>(static_cast<const cpx<double> *>(d_H), ld, d_n,
                                                                      batch, d_w, ldw, s, d_offsets));
        else
            LAUNCH("small_fused", s, launch_small_from_matrix<float>(static_cast<const cpx<float> *>(d_H), ld, d_n,
                                                                     batch, d_w, ldw, s, d_offsets));
        return MLMC_OK;
    }
    Carver cv{static_cast<char *>(d_work)};
    EigBuffers b;
    carve_large(cv, prec, ld, batch, false, b);
    return run_large(prec, d_H, ld, d_n, batch, d_w, ldw, b, s, false, false, d_offsets);
}

// Workspace of the banded eigenvector path (ld above the LDS-resident
// bound): a copy of the matrices for stage 1, the two-stage buffers, every
// panel's block reflector, the inverse iteration's LU factors and, for
// complex64 input, the vectors in complex128 until they are rounded.
struct EighLargeBuffers {
    EigBuffers b;
    double *w = nullptr;  // the bisection's eigenvalues [batch][ld]
    void *keep = nullptr;
    cpx<double> *tg = nullptr;  // the back-transformation's compound T factors
    void *ii = nullptr;
    cpx<double> *vd = nullptr;  // complex64 input: the vectors [batch][ld][ld] in complex128
};
static void carve_eigh_large(Carver &cv, mlmc_precision prec, int64_t ld, int64_t batch, EighLargeBuffers &L) {
    carve_large(cv, prec, ld, batch, true, L.b);
    L.w = cv.take<double>(sizeof(double) * (size_t)ld * (size_t)batch);
    L.keep = cv.take<void>(cplx_bytes(prec) * (size_t)eigh_keep_elems(ld) * (size_t)batch);
    L.tg = cv.take<cpx<double>>(sizeof(cpx<double>) * (size_t)eigh_group_t_elems(ld) * (size_t)batch);
    L.ii = cv.take<void>(band_ii_scratch_bytes(ld, batch));
    if (prec != MLMC_PREC_FP64) L.vd = cv.take<cpx<double>>(sizeof(cpx<double>) * (size_t)ld * (size_t)ld * (size_t)batch);
}

static mlmc_status eigh_workspace(mlmc_dtype dtype, mlmc_precision prec, int64_t ld, int64_t batch, size_t *bytes) {
    if (!bytes || ld < 0 || batch < 0) return fail(MLMC_ERR_INVALID_ARG, "eigh_workspace: bad argument");
    const mlmc_status st = check_dtype_prec(dtype, prec);
    if (st != MLMC_OK) return st;
    if (ld <= small_cap(prec)) {
        *bytes = eigh_work_bytes(ld, batch);
        return MLMC_OK;
    }
    if (ld > kEighLargeMax)
        return fail(MLMC_ERR_UNSUPPORTED, "batched_eigh: ld %lld exceeds %d", (long long)ld, kEighLargeMax);
    if (batch > 65535) return fail(MLMC_ERR_UNSUPPORTED, "batched_eigh: batch %lld above 65535 for ld > %d",
                                   (long long)batch, small_cap(prec));
    Carver cv{nullptr};
    EighLargeBuffers L;
    carve_eigh_large(cv, prec, ld, batch, L);
    *bytes = cv.used;
    return MLMC_OK;
}

extern "C++" {  // (a template, inside the C-linkage block of the entry points)
template <typename T>
static mlmc_status eigh_large(mlmc_precision prec, const void *d_H, int64_t ld, const int64_t *d_offsets,
                              const int32_t *d_n, int64_t batch, double *d_w, int64_t ldw, void *d_V, int64_t ldv,
                              void *d_work, hipStream_t s) {
    Carver cv{static_cast<char *>(d_work)};
    EighLargeBuffers L;
    carve_eigh_large(cv, prec, ld, batch, L);
    cpx<T> *Hc = static_cast<cpx<T> *>(L.b.H);
    cpx<T> *keep = static_cast<cpx<T> *>(L.keep);
    const int64_t keep_stride = eigh_keep_elems(ld);
    // complex128 vectors: the caller's buffer, or the workspace's copy for complex64 input
    cpx<double> *V = L.vd ? L.vd : static_cast<cpx<double> *>(d_V);
    const int64_t vld = L.vd ? ld : ldv;
    LAUNCH("eigh_gather", s, launch_gather_matrices<T>(static_cast<const cpx<T> *>(d_H), ld, d_offsets, d_n, batch, Hc, s));
    LAUNCH("band_reduce", s, launch_band_reduce_keep<T>(Hc, ld, d_n, batch, static_cast<cpx<T> *>(L.b.partial), s,
                                                        L.b.stride, nullptr, keep, keep_stride));
    mlmc_status rs = run_chase(prec, Hc, ld, d_n, batch, L.b, s);
    if (rs != MLMC_OK) return rs;
    rs = run_bisect(d_n, ld, batch, L.w, ld, L.b, s);
    if (rs != MLMC_OK) return rs;
    LAUNCH("eigh_band_ii", s, launch_band_inverse_iteration<T>(Hc, ld, d_n, batch, L.w, d_w, ldw, V, vld, L.ii, s));
    LAUNCH("eigh_backtransform", s, launch_panel_backtransform<T>(keep, keep_stride, ld, d_n, batch, V, vld, L.tg, s));
    if (L.vd)
        LAUNCH("eigh_narrow", s, launch_narrow_vectors(L.vd, ld, d_n, batch, static_cast<cpx<float> *>(d_V), ldv, s));
    return MLMC_OK;
}
}  // extern "C++"

// The eigenstates of validated arguments (d_work: eigh_workspace bytes).
static mlmc_status eigh_run(mlmc_precision prec, void *d_H, int64_t ld, const int64_t *d_offsets, const int32_t *d_n,
                            int64_t batch, double *d_w, int64_t ldw, void *d_V, int64_t ldv, void *d_work,
                            hipStream_t s) {
    if (ld <= small_cap(prec)) {
        if (prec == MLMC_PREC_FP64)
            LAUNCH("eigh_small", s, launch_eigh_small<double>(static_cast<const cpx<double> *>(d_H), ld, d_offsets,
                                                              d_n, batch, d_w, ldw, static_cast<cpx<double> *>(d_V),
                                                              ldv, static_cast<double *>(d_work), s));
        else
            LAUNCH("eigh_small", s, launch_eigh_small<float>(static_cast<const cpx<float> *>(d_H), ld, d_offsets,
                                                             d_n, batch, d_w, ldw, static_cast<cpx<float> *>(d_V),
                                                             ldv, static_cast<double *>(d_work), s));
        return MLMC_OK;
    }
    if (prec == MLMC_PREC_FP64)
        return eigh_large<double>(prec, d_H, ld, d_offsets, d_n, batch, d_w, ldw, d_V, ldv, d_work, s);
    return eigh_large<float>(prec, d_H, ld, d_offsets, d_n, batch, d_w, ldw, d_V, ldv, d_work, s);
}

mlmc_status mlmc_batched_eigh(mlmc_dtype dtype, mlmc_precision prec, void *d_H, int64_t ld, const int64_t *d_offsets,
                              const int32_t *d_n, int64_t batch, double *d_w, int64_t ldw, void *d_V, int64_t ldv,
                              void *d_work, size_t work_bytes, mlmc_stream stream) {
    size_t need = 0;
    const mlmc_status st = eigh_workspace(dtype, prec, ld, batch, &need);
    if (st != MLMC_OK) return st;
    if (ldw < ld || ldv < ld)
        return fail(MLMC_ERR_INVALID_ARG, "batched_eigh: ldw %lld, ldv %lld < ld %lld", (long long)ldw,
                    (long long)ldv, (long long)ld);
    if (batch > 0 && (!d_H || !d_n || !d_w || !d_V)) return fail(MLMC_ERR_INVALID_ARG, "batched_eigh: NULL buffer");
    if (need > 0 && (!d_work || work_bytes < need))
        return fail(MLMC_ERR_WORKSPACE, "batched_eigh: workspace %zu < %zu bytes", work_bytes, need);
    if (batch == 0 || ld == 0) return MLMC_OK;
    return eigh_run(prec, d_H, ld, d_offsets, d_n, batch, d_w, ldw, d_V, ldv, d_work, static_cast<hipStream_t>(stream));
}

// Generalised eigenstates: the Cholesky reduction's workspace, then the
// eigenstates' (both aligned).
static mlmc_status eigh_generalized_workspace(mlmc_dtype dtype, mlmc_precision prec, int64_t ld, int64_t batch,
                                              size_t *bytes, size_t *gen_bytes) {
    if (!bytes || ld < 0 || batch < 0) return fail(MLMC_ERR_INVALID_ARG, "eigh_generalized_workspace: bad argument");
    const mlmc_status st = check_dtype_prec(dtype, prec);
    if (st != MLMC_OK) return st;
    if (ld > kGenMax)
        return fail(MLMC_ERR_UNSUPPORTED, "batched_eigh_generalized: ld %lld exceeds %d", (long long)ld, kGenMax);
    size_t eb = 0;
    const mlmc_status se = eigh_workspace(dtype, prec, ld, batch, &eb);
    if (se != MLMC_OK) return se;
    const size_t ge = prec == MLMC_PREC_FP64 ? generalized_work_elems<double>(ld) : generalized_work_elems<float>(ld);
    const size_t gb = align_up(cplx_bytes(prec) * ge * (size_t)batch);
    if (gen_bytes) *gen_bytes = gb;
    *bytes = gb + eb;
    return MLMC_OK;
}

mlmc_status mlmc_batched_eigh_generalized(mlmc_dtype dtype, mlmc_precision prec, void *d_H, void *d_S, int64_t ld,
                                          const int32_t *d_n, int64_t batch, double *d_w, int64_t ldw, void *d_V,
                                          int64_t ldv, void *d_work, size_t work_bytes, mlmc_stream stream) {
    size_t need = 0, gen = 0;
    const mlmc_status st = eigh_generalized_workspace(dtype, prec, ld, batch, &need, &gen);
    if (st != MLMC_OK) return st;
    if (ldw < ld || ldv < ld)
        return fail(MLMC_ERR_INVALID_ARG, "batched_eigh_generalized: ldw %lld, ldv %lld < ld %lld", (long long)ldw,
                    (long long)ldv, (long long)ld);
    if (batch > 0 && (!d_H || !d_S || !d_n || !d_w || !d_V))
        return fail(MLMC_ERR_INVALID_ARG, "batched_eigh_generalized: NULL buffer");
    if (need > 0 && (!d_work || work_bytes < need))
        return fail(MLMC_ERR_WORKSPACE, "batched_eigh_generalized: workspace %zu < %zu bytes", work_bytes, need);
    if (batch == 0 || ld == 0) return MLMC_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char *work = static_cast<char *>(d_work);
    if (prec == MLMC_PREC_FP64)
        LAUNCH("overlap_reduce", s, launch_cholesky_reduce<double>(static_cast<cpx<double> *>(d_H),
                                                                   static_cast<cpx<double> *>(d_S), ld, d_n, batch,
                                                                   reinterpret_cast<cpx<double> *>(work), s));
    else
        LAUNCH("overlap_reduce", s, launch_cholesky_reduce<float>(static_cast<cpx<float> *>(d_H),
                                                                  static_cast<cpx<float> *>(d_S), ld, d_n, batch,
                                                                  reinterpret_cast<cpx<float> *>(work), s));
    const mlmc_status se = eigh_run(prec, d_H, ld, nullptr, d_n, batch, d_w, ldw, d_V, ldv, work + gen, s);
    if (se != MLMC_OK) return se;
    if (prec == MLMC_PREC_FP64)
        LAUNCH("eigh_backsolve", s, launch_trsm_lh<double>(static_cast<const cpx<double> *>(d_S), ld, d_n, batch,
                                                           static_cast<cpx<double> *>(d_V), ldv, s));
    else
        LAUNCH("eigh_backsolve", s, launch_trsm_lh<float>(static_cast<const cpx<float> *>(d_S), ld, d_n, batch,
                                                          static_cast<cpx<float> *>(d_V), ldv, s));
    return MLMC_OK;
}

}  // extern "C"

namespace {

constexpr int kMaxDevices = 64;

// Device address of `scratch` on each device, looked up once per device with
// that device current (the only per-process state of the library besides
// the caller's handles; written once, then read only).
struct ScratchAddress {
    std::once_flag once;
    void *ptr = nullptr;
    hipError_t err = hipSuccess;
};
ScratchAddress g_scratch_addr[kMaxDevices];

hipError_t scratch_address(void **out) {
    int dev = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess) return err;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    ScratchAddress &a = g_scratch_addr[dev];
    std::call_once(a.once, [&a]() { a.err = hipGetSymbolAddress(&a.ptr, HIP_SYMBOL(scratch)); });
    if (a.err != hipSuccess) return a.err;
    *out = a.ptr;
    return hipSuccess;
}

}  // namespace

extern "C" {

mlmc_status mlmc_batched_eigvalsh_noalloc(mlmc_dtype dtype, mlmc_precision prec, void *d_H, int64_t ld,
                                          const int32_t *d_n, int64_t batch, double *d_w, int64_t ldw,
                                          mlmc_stream stream) {
    size_t one = 0;
    mlmc_status st = eigvalsh_workspace(dtype, prec, ld, 1, &one);
    if (st != MLMC_OK) return st;
    if (batch < 0) return fail(MLMC_ERR_INVALID_ARG, "batched_eigvalsh_noalloc: batch %lld", (long long)batch);
    if (ldw < ld)
        return fail(MLMC_ERR_INVALID_ARG, "batched_eigvalsh_noalloc: ldw %lld < ld %lld", (long long)ldw, (long long)ld);
    if (batch > 0 && (!d_H || !d_n || !d_w)) return fail(MLMC_ERR_INVALID_ARG, "batched_eigvalsh_noalloc: NULL buffer");
    if (one > kNoAllocScratchBytes)
        return fail(MLMC_ERR_UNSUPPORTED,
                    "batched_eigvalsh_noalloc: one matrix of side %lld needs %zu bytes of scratch, more than the "
                    "%zu bytes this entry point has", (long long)ld, one, kNoAllocScratchBytes);
    if (batch == 0 || ld == 0) return MLMC_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (one == 0) {  // LDS-resident path: no scratch
        if (prec == MLMC_PREC_FP64)
            LAUNCH("small_fused", s, launch_small_from_matrix<double>(static_cast<const cpx<double> *>(d_H), ld, d_n, batch, d_w, ldw, s));
        else
            LAUNCH("small_fused", s, launch_small_from_matrix<float>(static_cast<const cpx<float> *>(d_H), ld, d_n, batch, d_w, ldw, s));
        return MLMC_OK;
    }
    void *base = nullptr;
    HIP_TRY(scratch_address(&base), "batched_eigvalsh_noalloc: scratch address");
    // The largest number of matrices whose workspace fits the scratch.
    int64_t chunk = (int64_t)(kNoAllocScratchBytes / one);
    if (chunk > batch) chunk = batch;
    for (;;) {
        size_t need = 0;
        st = eigvalsh_workspace(dtype, prec, ld, chunk, &need);
        if (st != MLMC_OK) return st;
        if (need <= kNoAllocScratchBytes || chunk == 1) break;
        --chunk;
    }
    // Chunks run one after another on `stream`, so each reuses the scratch
    // after the previous one is done with it.  Nothing in the workspace has
    // to start at zero: every kernel writes what it later reads.
    const size_t esize = cplx_bytes(prec);
    for (int64_t u0 = 0; u0 < batch; u0 += chunk) {
        const int64_t units = (batch - u0 < chunk) ? (batch - u0) : chunk;
        Carver cv{static_cast<char *>(base)};
        EigBuffers b;
        carve_large(cv, prec, ld, units, false, b);
        char *H = static_cast<char *>(d_H) + (size_t)u0 * (size_t)ld * (size_t)ld * esize;
        st = run_large(prec, H, ld, d_n + u0, units, d_w + u0 * ldw, ldw, b, s);
        if (st != MLMC_OK) return st;
    }
    return MLMC_OK;
}

static mlmc_status generalized_workspace(mlmc_dtype dtype, mlmc_precision prec, int64_t ld, int64_t batch,
                                         size_t *bytes) {
    if (!bytes || ld < 0 || batch < 0) return fail(MLMC_ERR_INVALID_ARG, "generalized_workspace: bad argument");
    const mlmc_status st = check_dtype_prec(dtype, prec);
    if (st != MLMC_OK) return st;
    if (ld > kGenMax)
        return fail(MLMC_ERR_UNSUPPORTED, "generalized eigvalsh: ld %lld exceeds %d", (long long)ld, kGenMax);
    Carver cv{nullptr};
    EigBuffers b;
    carve_generalized(cv, prec, ld, batch, false, b);
    *bytes = cv.used;
    return MLMC_OK;
}

mlmc_status mlmc_batched_eigvalsh_generalized(mlmc_dtype dtype, mlmc_precision prec, void *d_H, void *d_S,
                                              int64_t ld, const int32_t *d_n, int64_t batch, double *d_w,
                                              int64_t ldw, void *d_work, size_t work_bytes, mlmc_stream stream) {
    size_t need = 0;
    const mlmc_status st = generalized_workspace(dtype, prec, ld, batch, &need);
    if (st != MLMC_OK) return st;
    if (ldw < ld) return fail(MLMC_ERR_INVALID_ARG, "eigvalsh_generalized: ldw %lld < ld %lld", (long long)ldw, (long long)ld);
    if (batch > 0 && (!d_H || !d_S || !d_n || !d_w)) return fail(MLMC_ERR_INVALID_ARG, "eigvalsh_generalized: NULL buffer");
    if (need > 0 && (!d_work || work_bytes < need))
        return fail(MLMC_ERR_WORKSPACE, "eigvalsh_generalized: workspace %zu < %zu bytes", work_bytes, need);
    if (batch == 0 || ld == 0) return MLMC_OK;
    Carver cv{static_cast<char *>(d_work)};
    EigBuffers b;
    carve_generalized(cv, prec, ld, batch, false, b);
    return run_generalized(prec, d_H, d_S, ld, d_n, batch, d_w, ldw, b, static_cast<hipStream_t>(stream));
}

mlmc_status mlmc_idos(const double *d_w, int64_t ldw, const int32_t *d_n, int64_t n_samples, int32_t n_k,
                      const double *d_kweight, double area, const double *d_eps, int32_t n_eps, double delta,
                      mlmc_smoother smoother, double *d_idos, mlmc_stream stream) {
    if (n_samples < 0 || n_k < 1 || n_eps < 0 || ldw < 0)
        return fail(MLMC_ERR_INVALID_ARG, "idos: bad sizes (n_samples %lld, n_k %d, n_eps %d)", (long long)n_samples, n_k,
                    n_eps);
    if (!(delta > 0.0) || !std::isfinite(delta)) return fail(MLMC_ERR_INVALID_ARG, "idos: delta = %g", delta);
    if (!(area > 0.0) || !std::isfinite(area)) return fail(MLMC_ERR_INVALID_ARG, "idos: area = %g", area);
    if (smoother != MLMC_SMOOTH_GAUSS && smoother != MLMC_SMOOTH_CUBIC)
        return fail(MLMC_ERR_INVALID_ARG, "idos: bad smoother");
    if (n_samples > 0 && n_eps > 0 && (!d_w || !d_n || !d_kweight || !d_eps || !d_idos))
        return fail(MLMC_ERR_INVALID_ARG, "idos: NULL buffer");
    LAUNCH("idos", static_cast<hipStream_t>(stream), launch_idos(d_w, ldw, d_n, n_samples, n_k, d_kweight, 1.0 / area, d_eps, n_eps, delta, (int)smoother, d_idos,
                        static_cast<hipStream_t>(stream)));
    return MLMC_OK;
}

mlmc_status mlmc_level_stats(const double *d_idos_fine, const double *d_idos_quarters, int64_t n_samples,
                             int32_t n_eps, double *d_stats, mlmc_stream stream) {
    if (n_samples < 0 || n_eps < 0) return fail(MLMC_ERR_INVALID_ARG, "level_stats: negative size");
    if (n_samples > 0 && n_eps > 0 && (!d_idos_fine || !d_stats))
        return fail(MLMC_ERR_INVALID_ARG, "level_stats: NULL buffer");
    LAUNCH("level_stats", static_cast<hipStream_t>(stream), launch_level_stats(d_idos_fine, d_idos_quarters, n_samples, n_eps, d_stats, static_cast<hipStream_t>(stream)));
    return MLMC_OK;
}

static mlmc_status check_level_args(mlmc_lattice lat, int32_t N, int32_t coupled, int32_t Kf, int32_t Kc,
                                    mlmc_precision prec, int32_t n_eps) {
    if (!valid_lattice(lat)) return fail(MLMC_ERR_INVALID_ARG, "level: NULL lattice");
    if (N < 1 || N > 4096) return fail(MLMC_ERR_INVALID_ARG, "level: N = %d", N);
    if (coupled != 0 && coupled != 1) return fail(MLMC_ERR_INVALID_ARG, "level: coupled must be 0 or 1");
    if (coupled && N % 2 != 0) return fail(MLMC_ERR_INVALID_ARG, "level: coupled level needs even N, got %d", N);
    if (Kf < 1 || Kf > 4096 || (coupled && (Kc < 1 || Kc > 4096)))
        return fail(MLMC_ERR_INVALID_ARG, "level: K_fine = %d, K_coarse = %d", Kf, Kc);
    if (n_eps < 1) return fail(MLMC_ERR_INVALID_ARG, "level: n_eps = %d", n_eps);
    if (prec != MLMC_PREC_FP64 && prec != MLMC_PREC_MIXED) return fail(MLMC_ERR_INVALID_ARG, "level: bad precision");
    const int64_t nmax = (int64_t)lat->dev.n_orb * N * N;
    if (nmax > large_cap(prec))
        return fail(MLMC_ERR_UNSUPPORTED, "level: %lld orbitals exceed the %d the library supports", (long long)nmax,
                    large_cap(prec));
    if (lat->dev.n_ovl > 0 && nmax > kGenMax)
        return fail(MLMC_ERR_UNSUPPORTED, "level: the overlap (generalised) path supports at most %d orbitals", kGenMax);
    return MLMC_OK;
}

static mlmc_status level_workspace(mlmc_lattice lat, int32_t N_fine, int32_t coupled, int32_t K_fine,
                                   int32_t K_coarse, mlmc_kgrid_kind kind, int64_t chunk_samples, mlmc_precision prec,
                                   int32_t n_eps, size_t *bytes, int sets = kLevelSets) {
    const mlmc_status st = check_level_args(lat, N_fine, coupled, K_fine, K_coarse, prec, n_eps);
    if (st != MLMC_OK) return st;
    if (!valid_kgrid_kind(kind)) return fail(MLMC_ERR_INVALID_ARG, "level_workspace: bad k-grid");
    if (chunk_samples < 1) return fail(MLMC_ERR_INVALID_ARG, "level_workspace: chunk_samples must be >= 1");
    *bytes = level_layout(lat, N_fine, coupled != 0, K_fine, K_coarse, kind, chunk_samples, prec, n_eps, nullptr, sets)
                 .bytes;
    return MLMC_OK;
}

mlmc_status mlmc_workspace_bytes(const mlmc_workspace_request *req, size_t *bytes) {
    if (!req || !bytes) return fail(MLMC_ERR_INVALID_ARG, "workspace_bytes: NULL argument");
    *bytes = 0;
    switch (req->op) {
        case MLMC_OP_BATCHED_EIGVALSH: return eigvalsh_workspace(req->dtype, req->prec, req->ld, req->batch, bytes);
        case MLMC_OP_BATCHED_EIGVALSH_GENERALIZED:
            return generalized_workspace(req->dtype, req->prec, req->ld, req->batch, bytes);
        case MLMC_OP_LEVEL_ESTIMATE:
            return level_workspace(req->lat, req->N_fine, req->coupled, req->K_fine, req->K_coarse, req->kgrid,
                                   req->chunk_samples, req->prec, req->n_eps, bytes);
        case MLMC_OP_LEVEL_OUTCOMES_SINGLE_PASS:
            return level_workspace(req->lat, req->N_fine, req->coupled, req->K_fine, req->K_coarse, req->kgrid,
                                   req->chunk_samples, req->prec, req->n_eps, bytes, 1);
        case MLMC_OP_BATCHED_EIGH: return eigh_workspace(req->dtype, req->prec, req->ld, req->batch, bytes);
        case MLMC_OP_BATCHED_EIGH_GENERALIZED:
            return eigh_generalized_workspace(req->dtype, req->prec, req->ld, req->batch, bytes, nullptr);
        default: return fail(MLMC_ERR_INVALID_ARG, "workspace_bytes: unknown operation %d", (int)req->op);
    }
}

}  // extern "C"

namespace {

// Streams and events of one level call: with a context, three streams
// ordered by the context's events; without one, everything on the caller's
// stream (then the event operations are no-ops).
struct LevelStreams {
    mlmc_context ctx;
    hipStream_t front, chase, back;
    hipError_t record(hipEvent_t ev, hipStream_t st) const { return ctx ? hipEventRecord(ev, st) : hipSuccess; }
    hipError_t wait(hipStream_t st, hipEvent_t ev) const { return ctx ? hipStreamWaitEvent(st, ev, 0) : hipSuccess; }
};

// Sets the thread's launch timer for the duration of a call.
struct TimerScope {
    explicit TimerScope(LaunchTimer *t) { t_timer = t; }
    ~TimerScope() { t_timer = nullptr; }
};

// One MLMC level over M outcomes (Sections 2.2 and 3.3): the outcomes are
// drawn (d_mask_in == NULL: seed, first_sample, p) or given (d_mask_in:
// [M][N][N][G]).  Adds the level sums to d_stats (if not NULL) and writes the
// per-outcome Y and Q_f rows to d_Y, d_Q (if not NULL).
mlmc_status level_run(mlmc_context ctx, mlmc_lattice lat, int32_t N, bool cpl, double p, int32_t Kf, int32_t Kc,
                      mlmc_kgrid_kind kind, uint64_t seed, int64_t first_sample, int64_t *d_first,
                      const uint8_t *d_mask_in,
                      int64_t M, const double *d_eps, int32_t n_eps, double delta, mlmc_smoother smoother,
                      mlmc_precision prec, double *d_stats, double *d_Y, double *d_Q, void *d_work,
                      size_t work_bytes, hipStream_t s, bool single_pass_ok = false) {
    // A call allowed a single pass takes all M outcomes at once with one
    // buffer set when the workspace holds that; otherwise chunks in turn
    // over kLevelSets sets.
    const bool single = single_pass_ok && d_work &&
                        level_layout(lat, N, cpl, Kf, Kc, kind, M, prec, n_eps, nullptr, 1).bytes <= work_bytes;
    const size_t one = level_layout(lat, N, cpl, Kf, Kc, kind, 1, prec, n_eps, nullptr, single ? 1 : kLevelSets).bytes;
    if (!d_work || work_bytes < one)
        return fail(MLMC_ERR_WORKSPACE, "level: workspace %zu < %zu bytes needed for one sample", work_bytes, one);
    if (ctx) {
        int dev = -1;
        HIP_TRY(hipGetDevice(&dev), "level: device");
        if (dev != ctx->device)
            return fail(MLMC_ERR_INVALID_ARG, "level: context of device %d used on device %d", ctx->device, dev);
    }
    int64_t mc = M;
    if (!single) {
        const size_t two = level_layout(lat, N, cpl, Kf, Kc, kind, 2, prec, n_eps, nullptr).bytes;
        const size_t per = two - one, fixed = one - per;
        mc = (int64_t)((work_bytes - fixed) / per) + 2;  // padding makes the estimate approximate
        if (mc > M) mc = M;
        if (mc < 1) mc = 1;
        while (mc > 1 && level_layout(lat, N, cpl, Kf, Kc, kind, mc, prec, n_eps, nullptr).bytes > work_bytes) --mc;
    }
    const int nsets = single ? 1 : kLevelSets;
    const LevelLayout L = level_layout(lat, N, cpl, Kf, Kc, kind, mc, prec, n_eps, static_cast<char *>(d_work), nsets);
    const int G = lat->dev.n_groups, h = N / 2;
    const uint64_t tag = ((uint64_t)lat->dev.lattice_id << 32) | (uint64_t)(uint32_t)N;
    const uint64_t thr = (uint64_t)std::floor(p * 9007199254740992.0);
    const double inv_area_f = 1.0 / ((double)N * N * lat->dev.cell_area);
    const double inv_area_c = cpl ? 1.0 / ((double)h * h * lat->dev.cell_area) : 0.0;
    const int nkf = kgrid_count(kind, Kf), nkc = cpl ? kgrid_count(kind, Kc) : 0;
    const int64_t ldf = (int64_t)lat->dev.n_orb * N * N, ldc = (int64_t)lat->dev.n_orb * h * h;
    const int64_t mask_bytes = (int64_t)N * N * G;
    // With a context, three streams: the caller's (front) samples, assembles
    // and reduces chunk c (on the two-stage path: stage 1 only); the chase
    // stream chases chunk c's bands on 3/4 of the CUs while the front goes on
    // with chunk c + 1; the back stream runs chunk c's bisection, IDoS and
    // level sums.  Matrices (two-stage path), k-grids, sizes, tridiagonals and
    // eigenvalues come in kLevelSets sets used in turn; the front waits until
    // the back has released a set before refilling it.  The sample masks and
    // the stage-1 workspace are the front's alone, the band workspace the
    // chase stream's, the per-sample IDoS the back stream's.
    std::unique_lock<std::mutex> lk;
    if (ctx) lk = std::unique_lock<std::mutex>(ctx->mu);
    const LevelStreams S{ctx, s, ctx ? ctx->sc : s, ctx ? ctx->s : s};
    TimerScope timer_scope(ctx && !ctx->timer.ev.empty() ? &ctx->timer : nullptr);
    bool overlapping = false;
    int set0 = 0;
    if (ctx) {
        LayoutKey key;
        key.work = d_work;
        key.mc = mc;
        key.nkf = nkf;
        key.nkc = nkc;
        key.n_orb = lat->dev.n_orb;
        key.n_groups = G;
        key.N = N;
        key.n_eps = n_eps;
        key.prec = (int)prec;
        key.cpl = cpl;
        key.gen = lat->dev.n_ovl > 0;
        key.sets = nsets;
        // The previous call's front part (masks, stage-1 workspace, the last
        // chunk's matrices) is complete before this call's front starts.
        HIP_TRY(hipStreamWaitEvent(s, ctx->ready, 0), "level: wait");
        // Same layout on another stream than the previous call: the caller
        // alternates streams, so the next call is likely to start beside this
        // one's last chunk, which then keeps the chase stream's share of the CUs.
        overlapping = key == ctx->last && s != ctx->last_stream;
        ctx->last_stream = s;
        if (!(key == ctx->last)) {
            // Another layout may overlap any of the previous call's buffers:
            // all sets count as released only after everything enqueued so far.
            ctx->last = LayoutKey{};
            HIP_TRY(hipEventRecord(ctx->begin, s), "level: event");
            HIP_TRY(hipStreamWaitEvent(ctx->s, ctx->begin, 0), "level: wait");
            for (int q = 0; q < kLevelSets; ++q) HIP_TRY(hipEventRecord(ctx->freed[q], ctx->s), "level: event");
            ctx->last = key;
            ctx->next_set = 0;
        }
        set0 = ctx->next_set % nsets;
    }
    // A call that fails part-way makes the next one on its context take the
    // path above, with the front and chase work it did enqueue covered by
    // `ready` and the back stream.
    struct FailGuard {
        mlmc_context ctx;
        hipStream_t s;
        bool ok = false;
        ~FailGuard() {
            if (ok || !ctx) return;
            ctx->last = LayoutKey{};
            (void)hipEventRecord(ctx->chased, ctx->sc);
            (void)hipStreamWaitEvent(ctx->s, ctx->chased, 0);
            (void)hipEventRecord(ctx->ready, s);
        }
    } guard{ctx, s};
    int next_set = set0;
    mlmc_status st = MLMC_OK;
    for (int64_t done = 0; done < M; done += mc) {
        const int64_t ns = (M - done < mc) ? (M - done) : mc;
        const int q = next_set;
        next_set = (q + 1) % nsets;
        if (ctx) {
            ctx->next_set = next_set;
            HIP_TRY(hipStreamWaitEvent(s, ctx->freed[q], 0), "level: wait");
        }
        LAUNCH("kgrid", s, launch_kgrid(kind, Kf, L.kf[q], L.kwf[q], s));
        if (cpl) LAUNCH("kgrid", s, launch_kgrid(kind, Kc, L.kc[q], L.kwc[q], s));
        const uint8_t *mask = L.mask;
        if (d_mask_in)
            mask = d_mask_in + done * mask_bytes;
        else
            LAUNCH("sample_vacancies", s,
                   launch_sample_vacancies(lat->dev, N, thr, seed, tag, first_sample + done, ns, L.mask, s, d_first));
        bool pend_f = false, pend_c = false, chase_f = false, chase_c = false;
        const EigBuffers bf = L.bf.set(q), bc = L.bc.set(q);
        const int upd = ctx ? ctx->upd_rows : 32;
        st = outcome_spectra(lat, N, mask, ns, L.kf[q], nkf, prec, L.wf[q], L.nf[q], bf, s, &pend_f, &chase_f, upd);
        if (st != MLMC_OK) return st;
        if (cpl) {
            LAUNCH("partition", s, launch_partition(N, G, mask, ns, L.quarters, s));
            st = outcome_spectra(lat, h, L.quarters, ns * 4, L.kc[q], nkc, prec, L.wc[q], L.nc[q], bc, s, &pend_c,
                                 &chase_c, upd);
            if (st != MLMC_OK) return st;
        }
        hipStream_t sc = S.chase, sb = S.back;
        if (ctx) {
            HIP_TRY(hipEventRecord(ctx->ready, s), "level: event");
            HIP_TRY(hipStreamWaitEvent(sb, ctx->ready, 0), "level: wait");
        }
        // The last chunk's chase and bisection have nothing left to run
        // beside (unless the calls overlap): they take the whole device (one
        // workgroup per matrix), as does everything without a context.
        const bool last = !ctx || (!overlapping && done + ns >= M);
        const int64_t chase_blocks = last ? 0 : ctx->chase_blocks, bisect_blocks = last ? 0 : ctx->bisect_blocks;
        if (chase_f || chase_c) {
            if (ctx) HIP_TRY(hipStreamWaitEvent(sc, ctx->ready, 0), "level: wait");
            if (chase_f) {
                st = run_chase(prec, bf.H, ldf, L.nf[q], ns * nkf, bf, sc, chase_blocks);
                if (st != MLMC_OK) return st;
            }
            if (chase_c) {
                st = run_chase(prec, bc.H, ldc, L.nc[q], ns * 4 * nkc, bc, sc, chase_blocks);
                if (st != MLMC_OK) return st;
            }
            if (ctx) {
                HIP_TRY(hipEventRecord(ctx->chased, sc), "level: event");
                HIP_TRY(hipStreamWaitEvent(sb, ctx->chased, 0), "level: wait");
            }
        }
        if (pend_f) {
            st = run_bisect(L.nf[q], ldf, ns * nkf, L.wf[q], ldf, bf, sb, bisect_blocks);
            if (st != MLMC_OK) return st;
        }
        LAUNCH("idos", sb, launch_idos(L.wf[q], ldf, L.nf[q], ns, nkf, L.kwf[q], inv_area_f, d_eps, n_eps, delta,
                                       (int)smoother, L.If, sb));
        if (cpl) {
            if (pend_c) {
                st = run_bisect(L.nc[q], ldc, ns * 4 * nkc, L.wc[q], ldc, bc, sb, bisect_blocks);
                if (st != MLMC_OK) return st;
            }
            LAUNCH("idos", sb, launch_idos(L.wc[q], ldc, L.nc[q], ns * 4, nkc, L.kwc[q], inv_area_c, d_eps, n_eps,
                                           delta, (int)smoother, L.Ic, sb));
        }
        LAUNCH("level_stats", sb,
               launch_level_stats(L.If, cpl ? L.Ic : nullptr, ns, n_eps, d_stats, sb,
                                  d_Y ? d_Y + done * n_eps : nullptr, d_Q ? d_Q + done * n_eps : nullptr));
        if (ctx) HIP_TRY(hipEventRecord(ctx->freed[q], sb), "level: event");
    }
    // the device-resident counter moves past this call's samples (after the
    // last sampling kernel, which ran on this stream)
    if (d_first) HIP_TRY(launch_advance_counter(d_first, M, s), "level: counter");
    guard.ok = true;
    if (ctx) {
        HIP_TRY(hipEventRecord(ctx->end, ctx->s), "level: event");
        HIP_TRY(hipStreamWaitEvent(s, ctx->end, 0), "level: wait");
    }
    return MLMC_OK;
}

mlmc_status check_level_call(mlmc_lattice lat, int32_t N, int32_t coupled, double p, int32_t Kf, int32_t Kc,
                             mlmc_kgrid_kind kind, int64_t M, const double *d_eps, int32_t n_eps, double delta,
                             mlmc_smoother smoother, mlmc_precision prec) {
    mlmc_status st = check_level_args(lat, N, coupled, Kf, Kc, prec, n_eps);
    if (st != MLMC_OK) return st;
    if (!(p >= 0.0 && p <= 1.0)) return fail(MLMC_ERR_INVALID_ARG, "level: p = %g", p);
    if (!(delta > 0.0) || !std::isfinite(delta)) return fail(MLMC_ERR_INVALID_ARG, "level: delta = %g", delta);
    if (!valid_kgrid_kind(kind)) return fail(MLMC_ERR_INVALID_ARG, "level: bad k-grid");
    if (smoother != MLMC_SMOOTH_GAUSS && smoother != MLMC_SMOOTH_CUBIC)
        return fail(MLMC_ERR_INVALID_ARG, "level: bad smoother");
    if (M < 0) return fail(MLMC_ERR_INVALID_ARG, "level: negative sample count");
    if (M > 0 && !d_eps) return fail(MLMC_ERR_INVALID_ARG, "level: NULL energies");
    return MLMC_OK;
}

}  // namespace

extern "C" {

mlmc_status mlmc_level_estimate(mlmc_lattice lat, int32_t N, int32_t coupled, double p, int32_t Kf, int32_t Kc,
                                mlmc_kgrid_kind kind, uint64_t seed, int64_t first_sample, int64_t M,
                                const double *d_eps, int32_t n_eps, double delta, mlmc_smoother smoother,
                                mlmc_precision prec, double *d_stats, void *d_work, size_t work_bytes,
                                int64_t *d_first_sample, mlmc_context ctx, mlmc_stream stream) {
    mlmc_status st = check_level_call(lat, N, coupled, p, Kf, Kc, kind, M, d_eps, n_eps, delta, smoother, prec);
    if (st != MLMC_OK) return st;
    if (first_sample < 0) return fail(MLMC_ERR_INVALID_ARG, "level: negative first sample");
    if (M == 0) return MLMC_OK;
    if (!d_stats) return fail(MLMC_ERR_INVALID_ARG, "level: NULL stats");
    return level_run(ctx, lat, N, coupled != 0, p, Kf, Kc, kind, seed, first_sample, d_first_sample, nullptr, M, d_eps,
                     n_eps, delta, smoother, prec, d_stats, nullptr, nullptr, d_work, work_bytes,
                     static_cast<hipStream_t>(stream));
}

mlmc_status mlmc_level_outcomes(mlmc_lattice lat, int32_t N, int32_t coupled, int32_t Kf, int32_t Kc,
                                mlmc_kgrid_kind kind, const uint8_t *d_mask, int64_t M, const double *d_eps,
                                int32_t n_eps, double delta, mlmc_smoother smoother, mlmc_precision prec,
                                double *d_stats, double *d_Y, double *d_Q, void *d_work, size_t work_bytes,
                                mlmc_context ctx, mlmc_stream stream) {
    mlmc_status st = check_level_call(lat, N, coupled, 0.0, Kf, Kc, kind, M, d_eps, n_eps, delta, smoother, prec);
    if (st != MLMC_OK) return st;
    if (M == 0) return MLMC_OK;
    if (!d_mask) return fail(MLMC_ERR_INVALID_ARG, "level_outcomes: NULL mask");
    if (!d_stats && !d_Y && !d_Q) return fail(MLMC_ERR_INVALID_ARG, "level_outcomes: no output");
    return level_run(ctx, lat, N, coupled != 0, 0.0, Kf, Kc, kind, 0, 0, nullptr, d_mask, M, d_eps, n_eps, delta, smoother,
                     prec, d_stats, d_Y, d_Q, d_work, work_bytes, static_cast<hipStream_t>(stream), true);
}

mlmc_status mlmc_context_create(mlmc_context *out) {
    if (!out) return fail(MLMC_ERR_INVALID_ARG, "context_create: NULL argument");
    *out = nullptr;
    auto *c = new mlmc_context_s();
    hipError_t err = hipGetDevice(&c->device);
    int cus = 0;
    if (err == hipSuccess) err = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device);
    // One bisection workgroup per CU leaves the rest of each CU to the next
    // chunk's reduction on the caller's stream (measured best among 1/4 to 8
    // per CU on the graphene N = 16 workload).
    c->bisect_blocks = cus > 0 ? cus : 1;
    c->chase_blocks = chase_cus(cus);
    // Default-priority streams that do not synchronise with the null stream,
    // created one after another: the runtime spreads consecutively created
    // streams over its hardware queues, so the two caller streams, the back
    // stream and the chase stream do not share one (streams that share a
    // hardware queue run their work in order, which would serialise the
    // chase behind the next chunk's reduction).
    if (err == hipSuccess) err = hipStreamCreateWithFlags(&c->front[0], hipStreamNonBlocking);
    if (err == hipSuccess) err = hipStreamCreateWithFlags(&c->front[1], hipStreamNonBlocking);
    if (err == hipSuccess) err = hipStreamCreateWithFlags(&c->s, hipStreamNonBlocking);
    if (err == hipSuccess) err = hipStreamCreateWithFlags(&c->sc, hipStreamNonBlocking);
    hipEvent_t *evs[4 + kLevelSets] = {&c->begin, &c->ready, &c->chased, &c->end};
    for (int q = 0; q < kLevelSets; ++q) evs[4 + q] = &c->freed[q];
    for (hipEvent_t *ev : evs)
        if (err == hipSuccess) err = hipEventCreateWithFlags(ev, hipEventDisableTiming);
    // Every event a level estimate waits for has been recorded at least once.
    if (err == hipSuccess) err = hipEventRecord(c->ready, c->s);
    if (err == hipSuccess) err = hipEventRecord(c->chased, c->s);
    if (err != hipSuccess) {
        (void)c->release();
        delete c;
        return hip_fail(err, "context_create");
    }
    *out = c;
    return MLMC_OK;
}

mlmc_status mlmc_context_destroy(mlmc_context ctx) {
    if (!ctx) return MLMC_OK;
    hipError_t err;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        int prev = -1;
        err = hipGetDevice(&prev);
        if (err == hipSuccess && prev != ctx->device) err = hipSetDevice(ctx->device);
        const hipError_t e2 = ctx->release();
        if (err == hipSuccess) err = e2;
        if (prev >= 0 && prev != ctx->device) (void)hipSetDevice(prev);
    }
    delete ctx;
    if (err != hipSuccess) return hip_fail(err, "context_destroy");
    return MLMC_OK;
}

mlmc_status mlmc_context_stream(mlmc_context ctx, int32_t index, mlmc_stream *out) {
    if (!ctx || !out || index < 0 || index > 1) return fail(MLMC_ERR_INVALID_ARG, "context_stream: bad argument");
    *out = ctx->front[index];
    return MLMC_OK;
}

mlmc_status mlmc_context_configure(mlmc_context ctx, const mlmc_launch_config *cfg) {
    if (!ctx || !cfg) return fail(MLMC_ERR_INVALID_ARG, "context_configure: NULL argument");
    if (cfg->chase_workgroups < 0 || cfg->bisect_workgroups < 0)
        return fail(MLMC_ERR_INVALID_ARG, "context_configure: negative workgroup count");
    if (cfg->update_tile_rows != 0 && cfg->update_tile_rows != 32 && cfg->update_tile_rows != 64)
        return fail(MLMC_ERR_INVALID_ARG, "context_configure: update_tile_rows %d (0, 32 or 64)",
                    (int)cfg->update_tile_rows);
    int cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device), "context_configure");
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->chase_blocks = cfg->chase_workgroups > 0 ? cfg->chase_workgroups : chase_cus(cus);
    ctx->bisect_blocks = cfg->bisect_workgroups > 0 ? cfg->bisect_workgroups : (cus > 0 ? cus : 1);
    ctx->upd_rows = cfg->update_tile_rows > 0 ? cfg->update_tile_rows : 32;
    return MLMC_OK;
}

mlmc_status mlmc_context_timer(mlmc_context ctx, int64_t capacity, int32_t detail) {
    if (!ctx || capacity < 0 || capacity > (int64_t)1 << 20)
        return fail(MLMC_ERR_INVALID_ARG, "context_timer: bad argument");
    std::lock_guard<std::mutex> lk(ctx->mu);
    LaunchTimer &t = ctx->timer;
    t.detail = detail != 0;
    if ((int64_t)t.names.size() == capacity) {  // same capacity: keep the events, forget the records
        t.used = 0;
        t.dropped = 0;
        return MLMC_OK;
    }
    t.release();
    if (capacity == 0) return MLMC_OK;
    t.ev.assign(2 * (size_t)capacity, nullptr);
    t.names.assign((size_t)capacity, nullptr);
    for (hipEvent_t &e : t.ev) {
        const hipError_t err = hipEventCreate(&e);
        if (err != hipSuccess) {
            t.release();
            return hip_fail(err, "context_timer");
        }
    }
    return MLMC_OK;
}

mlmc_status mlmc_context_timer_read(mlmc_context ctx, const char *name, double *total_ms, int64_t *launches,
                                    int64_t *dropped) {
    if (!ctx || !name || !total_ms || !launches) return fail(MLMC_ERR_INVALID_ARG, "context_timer_read: NULL argument");
    std::lock_guard<std::mutex> lk(ctx->mu);
    const LaunchTimer &t = ctx->timer;
    double total = 0.0;
    int64_t count = 0;
    for (size_t r = 0; r < t.used; ++r) {
        if (!t.names[r] || std::strcmp(t.names[r], name) != 0) continue;
        HIP_TRY(hipEventSynchronize(t.ev[2 * r + 1]), "timer_read");
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, t.ev[2 * r], t.ev[2 * r + 1]), "timer_read");
        total += ms;
        ++count;
    }
    *total_ms = total;
    *launches = count;
    if (dropped) *dropped = t.dropped;
    return MLMC_OK;
}

mlmc_status mlmc_chase_cus(mlmc_precision prec, int64_t *cus) {
    if (!cus) return fail(MLMC_ERR_INVALID_ARG, "chase_cus: NULL argument");
    if (prec != MLMC_PREC_FP64 && prec != MLMC_PREC_MIXED) return fail(MLMC_ERR_INVALID_ARG, "chase_cus: bad prec");
    int dev = 0, n = 0;
    HIP_TRY(hipGetDevice(&dev), "chase_cus: device");
    HIP_TRY(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev), "chase_cus: attribute");
    *cus = chase_cus(n);
    return MLMC_OK;
}

mlmc_status mlmc_dos(int32_t n_eps, const double *eps, const double *idos, double *dos) {
    if (n_eps < 3 || !eps || !idos || !dos) return fail(MLMC_ERR_INVALID_ARG, "dos: need n_eps >= 3 and buffers");
    for (int j = 1; j < n_eps; ++j)
        if (!(eps[j] > eps[j - 1])) return fail(MLMC_ERR_INVALID_ARG, "dos: eps not increasing at %d", j);
    // f'(x1) from f(x0), f(x1), f(x2) with a = x1 - x0, b = x2 - x1: exact for quadratics
    for (int j = 1; j + 1 < n_eps; ++j) {
        const double a = eps[j] - eps[j - 1], b = eps[j + 1] - eps[j];
        dos[j] = (-b / (a * (a + b))) * idos[j - 1] + ((b - a) / (a * b)) * idos[j] + (a / (b * (a + b))) * idos[j + 1];
    }
    {
        const double a = eps[1] - eps[0], b = eps[2] - eps[1];
        dos[0] = (-(2.0 * a + b) / (a * (a + b))) * idos[0] + ((a + b) / (a * b)) * idos[1] - (a / (b * (a + b))) * idos[2];
    }
    {
        const int k = n_eps - 1;
        const double a = eps[k - 1] - eps[k - 2], b = eps[k] - eps[k - 1];
        dos[k] = (b / (a * (a + b))) * idos[k - 2] - ((a + b) / (a * b)) * idos[k - 1] + ((2.0 * b + a) / (b * (a + b))) * idos[k];
    }
    return MLMC_OK;
}

mlmc_status mlmc_optimal_samples(int32_t L, const double *V, const double *W, double C_alpha, double theta, double tol,
                                 double *M_out) {
    if (L < 1 || !V || !W || !M_out) return fail(MLMC_ERR_INVALID_ARG, "optimal_samples: bad argument");
    if (!(theta > 0.0) || !(tol > 0.0) || !(C_alpha > 0.0))
        return fail(MLMC_ERR_INVALID_ARG, "optimal_samples: theta, tol and C_alpha must be > 0");
    double total = 0.0;
    for (int l = 0; l < L; ++l) {
        if (!(V[l] >= 0.0) || !(W[l] > 0.0)) return fail(MLMC_ERR_INVALID_ARG, "optimal_samples: V[%d], W[%d]", l, l);
        total += std::sqrt(W[l] * V[l]);
    }
    const double scale = (C_alpha / (theta * tol)) * (C_alpha / (theta * tol));
    for (int l = 0; l < L; ++l) M_out[l] = scale * std::sqrt(V[l] / W[l]) * total;
    return MLMC_OK;
}

}  // extern "C"


