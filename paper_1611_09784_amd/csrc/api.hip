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

#include "internal.hpp"

using namespace mlmc;

struct mlmc_lattice_s {
    int device = -1;
    DevLattice dev{};
    void *d_buf = nullptr;
};

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

// Opt-in launch timing (mlmc_timer_enable / mlmc_timer_read): a start/stop
// event pair recorded on the launch stream around each kernel launch.
struct TimerRec {
    const char *name;
    hipEvent_t start, stop;
};
std::mutex g_timer_mu;
std::atomic<bool> g_timing{false};
std::vector<TimerRec> g_timer_recs;

void timer_clear_locked() {
    for (auto &r : g_timer_recs) {
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    g_timer_recs.clear();
}

template <typename F>
hipError_t timed(const char *name, hipStream_t s, F &&launch) {
    if (!g_timing.load(std::memory_order_relaxed)) return launch();
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t err = hipEventCreate(&a);
    if (err == hipSuccess) err = hipEventCreate(&b);
    if (err == hipSuccess) err = hipEventRecord(a, s);
    if (err != hipSuccess) return err;
    err = launch();
    const hipError_t e2 = hipEventRecord(b, s);
    {
        std::lock_guard<std::mutex> lk(g_timer_mu);
        g_timer_recs.push_back({name, a, b});
    }
    return err != hipSuccess ? err : e2;
}

#define LAUNCH(name, stream, expr) HIP_TRY(timed(name, stream, [&]() { return (expr); }), name)

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
                      const EigBuffers &b, hipStream_t s, int64_t max_blocks = 0) {
    if (prec == MLMC_PREC_FP64)
        LAUNCH("chase", s, launch_band_chase<double>(static_cast<const cpx<double> *>(H), ld, n, units, b.d, b.e, ld,
                                                     static_cast<cpx<double> *>(b.partial), s, max_blocks, b.stride));
    else
        LAUNCH("chase", s, launch_band_chase<float>(static_cast<const cpx<float> *>(H), ld, n, units, b.d, b.e, ld,
                                                    static_cast<cpx<float> *>(b.partial), s, max_blocks, b.stride));
    return MLMC_OK;
}

// With defer_chase only stage 1 runs here (the caller runs run_chase and
// run_bisect, possibly on other streams).
mlmc_status run_large(mlmc_precision prec, void *H, int64_t ld, const int32_t *n, int64_t units, double *w, int64_t ldw,
                      const EigBuffers &b, hipStream_t s, bool defer_bisect = false, bool defer_chase = false) {
    if (prec == MLMC_PREC_FP64)
        LAUNCH("band_reduce", s, launch_band_reduce<double>(static_cast<cpx<double> *>(H), ld, n, units,
                                                            static_cast<cpx<double> *>(b.partial), s, b.stride));
    else
        LAUNCH("band_reduce", s, launch_band_reduce<float>(static_cast<cpx<float> *>(H), ld, n, units,
                                                           static_cast<cpx<float> *>(b.partial), s, b.stride));
    if (defer_chase) return MLMC_OK;
    const mlmc_status st = run_chase(prec, H, ld, n, units, b, s);
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
    size_t bytes = 0;
};

static bool valid_kgrid_kind(int kind) {
    return kind == MLMC_KGRID_MP || kind == MLMC_KGRID_GAMMA || kind == MLMC_KGRID_RHOMBI;
}

LevelLayout level_layout(const mlmc_lattice_s *lat, int N, bool coupled, int Kf, int Kc, int kind, int64_t mc,
                         mlmc_precision prec, int n_eps, char *base) {
    LevelLayout L;
    Carver cv{base};
    const int G = lat->dev.n_groups, no = lat->dev.n_orb;
    const int64_t nkf = kgrid_count(kind, Kf), nkc = kgrid_count(kind, Kc);
    const int64_t ldf = (int64_t)no * N * N;
    for (int q = 0; q < kLevelSets; ++q) {
        L.kf[q] = cv.take<double>(sizeof(double) * 2 * nkf);
        L.kwf[q] = cv.take<double>(sizeof(double) * nkf);
    }
    L.mask = cv.take<uint8_t>((size_t)mc * N * N * G);
    for (int q = 0; q < kLevelSets; ++q) {
        L.nf[q] = cv.take<int32_t>(sizeof(int32_t) * (size_t)(mc * nkf));
        L.wf[q] = cv.take<double>(sizeof(double) * (size_t)(mc * nkf * ldf));
    }
    L.If = cv.take<double>(sizeof(double) * (size_t)mc * n_eps);
    const bool gen = lat->dev.n_ovl > 0;
    if (gen) carve_generalized(cv, prec, ldf, mc * nkf, true, L.bf, kLevelSets);
    else if (ldf > small_cap(prec)) carve_large(cv, prec, ldf, mc * nkf, true, L.bf, kLevelSets);
    if (coupled) {
        const int h = N / 2;
        const int64_t ldc = (int64_t)no * h * h;
        for (int q = 0; q < kLevelSets; ++q) {
            L.kc[q] = cv.take<double>(sizeof(double) * 2 * nkc);
            L.kwc[q] = cv.take<double>(sizeof(double) * nkc);
        }
        L.quarters = cv.take<uint8_t>((size_t)mc * 4 * h * h * G);
        for (int q = 0; q < kLevelSets; ++q) {
            L.nc[q] = cv.take<int32_t>(sizeof(int32_t) * (size_t)(mc * 4 * nkc));
            L.wc[q] = cv.take<double>(sizeof(double) * (size_t)(mc * 4 * nkc * ldc));
        }
        L.Ic = cv.take<double>(sizeof(double) * (size_t)mc * 4 * n_eps);
        if (gen) carve_generalized(cv, prec, ldc, mc * 4 * nkc, true, L.bc, kLevelSets);
        else if (ldc > small_cap(prec)) carve_large(cv, prec, ldc, mc * 4 * nkc, true, L.bc, kLevelSets);
    }
    L.bytes = cv.used;
    return L;
}

// Pencils (H, S) already in b.H, b.S -> eigenvalues (reduction to C = L^{-1}
// H L^{-H}, then the standard path on C).
mlmc_status run_generalized(mlmc_precision prec, void *H, void *S, int64_t ld, const int32_t *n, int64_t units,
                            double *w, int64_t ldw, const EigBuffers &b, hipStream_t s, bool *bisect_pending = nullptr,
                            bool *chase_pending = nullptr) {
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
                     bisect_pending != nullptr && chase_pending != nullptr);
}

// Eigenvalues of every (outcome, k) unit of `ns` outcomes of side N.  With
// bisect_pending, a path that ends in a bisection stops before it and says so
// (the caller then calls run_bisect on the same buffers); with chase_pending
// as well, the two-stage path stops after stage 1 (the caller then calls
// run_chase first).
mlmc_status outcome_spectra(const mlmc_lattice_s *lat, int N, const uint8_t *mask, int64_t ns, const double *kred,
                            int nk, mlmc_precision prec, double *w, int32_t *n_out, const EigBuffers &b,
                            hipStream_t s, bool *bisect_pending = nullptr, bool *chase_pending = nullptr) {
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
        return run_generalized(prec, b.H, b.S, ld, n_out, units, w, ld, b, s, bisect_pending, chase_pending);
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
                     bisect_pending != nullptr && chase_pending != nullptr);
}

// The library's two streams on the current device (back: bisection, IDoS,
// level sums; chase), with the events that order them against the caller's
// stream in mlmc_level_estimate.  Created on first use, default priority;
// kept until the process ends.
struct BackStream {
    hipStream_t s = nullptr;
    hipStream_t sc = nullptr;     // the chase stream
    int64_t bisect_blocks = 0;    // workgroups of a bisection on the back stream: one per CU
    int64_t chase_blocks = 0;     // workgroups of a chase on the chase stream
    hipEvent_t begin = nullptr;   // caller's stream -> back stream
    hipEvent_t ready = nullptr;   // front (caller's stream) -> chase and back: a chunk's front part is complete
    hipEvent_t chased = nullptr;  // chase -> back: a chunk's tridiagonals are complete
    hipEvent_t freed[kLevelSets] = {};  // back -> front: set q of the matrices / sizes / tridiagonals /
                                        // eigenvalues is free
    hipEvent_t end = nullptr;     // back -> caller's stream
    bool created = false;         // streams and events all created
    // The previous level estimate's workspace layout and the set its next
    // chunk would use.  A call with the same layout continues the rotation:
    // each of its chunks waits only for the release of its own set (and its
    // first for the previous call's front part), so it may start while the
    // previous call's last chunks are still chased and bisected.
    struct LayoutKey {
        const void *work = nullptr;
        int64_t mc = 0, nkf = 0, nkc = 0;
        int n_orb = 0, n_groups = 0, N = 0, n_eps = 0, prec = 0;
        bool cpl = false, gen = false;
        bool operator==(const LayoutKey &o) const {
            return work == o.work && mc == o.mc && nkf == o.nkf && nkc == o.nkc && n_orb == o.n_orb &&
                   n_groups == o.n_groups && N == o.N && n_eps == o.n_eps && prec == o.prec && cpl == o.cpl &&
                   gen == o.gen;
        }
    } last;
    int next_set = 0;
    hipStream_t last_stream = nullptr;  // the previous call's stream
};
constexpr int kMaxDevices = 64;
std::mutex g_back_mu;  // held while a level estimate enqueues its work

// Workgroups (one per CU) of a chase on the chase stream: the next chunk's
// stage 1 runs on the quarter of the CUs it leaves free and, with the 32-row
// rank-2k update, beside it on the others (measured on the graphene N = 16
// workload: FP64 3/4 of the CUs 24.7k eigensolves/s, 5/8 22.9k, 7/8 24.1k,
// all 21.9k; mixed 40.3k, 37.6k, 38.8k, 30.1k).
int64_t chase_cus(int cus) {
    const int64_t v = (int64_t)cus * 3 / 4;
    return v > 0 ? v : 1;
}
BackStream g_back[kMaxDevices];

hipError_t back_stream(BackStream **out) {
    int dev = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess) return err;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    BackStream &b = g_back[dev];
    if (!b.created) {
        // One bisection workgroup per CU leaves the rest of each CU to the
        // next chunk's reduction on the caller's stream (measured best among
        // 1/4 to 8 per CU on the graphene N = 16 workload).
        int cus = 0;
        err = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (err != hipSuccess) return err;
        b.bisect_blocks = cus > 0 ? cus : 1;
        b.chase_blocks = chase_cus(cus);
        // (What a failed attempt did create is kept and the rest tried again.)
        if (!b.s) err = hipStreamCreateWithFlags(&b.s, hipStreamNonBlocking);
        if (err == hipSuccess && !b.sc) err = hipStreamCreateWithFlags(&b.sc, hipStreamNonBlocking);
        hipEvent_t *evs[4 + kLevelSets] = {&b.begin, &b.ready, &b.chased, &b.end};
        for (int q = 0; q < kLevelSets; ++q) evs[4 + q] = &b.freed[q];
        for (hipEvent_t *ev : evs)
            if (err == hipSuccess && !*ev) err = hipEventCreateWithFlags(ev, hipEventDisableTiming);
        // Every event a level estimate waits for has been recorded at least once.
        if (err == hipSuccess) err = hipEventRecord(b.ready, b.s);
        if (err == hipSuccess) err = hipEventRecord(b.chased, b.s);
        if (err != hipSuccess) return err;
        b.created = true;
    }
    *out = &b;
    return hipSuccess;
}

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

mlmc_status mlmc_eigvalsh_workspace(mlmc_dtype dtype, mlmc_precision prec, int64_t ld, int64_t batch, size_t *bytes) {
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

mlmc_status mlmc_batched_eigvalsh(mlmc_dtype dtype, mlmc_precision prec, void *d_H, int64_t ld, const int32_t *d_n,
                                  int64_t batch, double *d_w, int64_t ldw, void *d_work, size_t work_bytes,
                                  mlmc_stream stream) {
    size_t need = 0;
    const mlmc_status st = mlmc_eigvalsh_workspace(dtype, prec, ld, batch, &need);
    if (st != MLMC_OK) return st;
    if (ldw < ld) return fail(MLMC_ERR_INVALID_ARG, "batched_eigvalsh: ldw %lld < ld %lld", (long long)ldw, (long long)ld);
    if (batch > 0 && (!d_H || !d_n || !d_w)) return fail(MLMC_ERR_INVALID_ARG, "batched_eigvalsh: NULL buffer");
    if (need > 0 && (!d_work || work_bytes < need))
        return fail(MLMC_ERR_WORKSPACE, "batched_eigvalsh: workspace %zu < %zu bytes", work_bytes, need);
    if (batch == 0 || ld == 0) return MLMC_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (ld <= small_cap(prec)) {
        if (prec == MLMC_PREC_FP64)
            LAUNCH("small_fused", s, launch_small_from_matrix<double>(static_cast<const cpx<double> *>(d_H), ld, d_n, batch, d_w, ldw, s));
        else
            LAUNCH("small_fused", s, launch_small_from_matrix<float>(static_cast<const cpx<float> *>(d_H), ld, d_n, batch, d_w, ldw, s));
        return MLMC_OK;
    }
    Carver cv{static_cast<char *>(d_work)};
    EigBuffers b;
    carve_large(cv, prec, ld, batch, false, b);
    return run_large(prec, d_H, ld, d_n, batch, d_w, ldw, b, s);
}

mlmc_status mlmc_generalized_workspace(mlmc_dtype dtype, mlmc_precision prec, int64_t ld, int64_t batch,
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
    const mlmc_status st = mlmc_generalized_workspace(dtype, prec, ld, batch, &need);
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

mlmc_status mlmc_level_workspace(mlmc_lattice lat, int32_t N_fine, int32_t coupled, int32_t K_fine, int32_t K_coarse,
                                 mlmc_kgrid_kind kind, int64_t chunk_samples, mlmc_precision prec, int32_t n_eps,
                                 size_t *bytes) {
    const mlmc_status st = check_level_args(lat, N_fine, coupled, K_fine, K_coarse, prec, n_eps);
    if (st != MLMC_OK) return st;
    if (!valid_kgrid_kind(kind)) return fail(MLMC_ERR_INVALID_ARG, "level_workspace: bad k-grid");
    if (!bytes || chunk_samples < 1) return fail(MLMC_ERR_INVALID_ARG, "level_workspace: chunk_samples must be >= 1");
    *bytes = level_layout(lat, N_fine, coupled != 0, K_fine, K_coarse, kind, chunk_samples, prec, n_eps, nullptr).bytes;
    return MLMC_OK;
}

mlmc_status mlmc_level_estimate(mlmc_lattice lat, int32_t N, int32_t coupled, double p, int32_t Kf, int32_t Kc,
                                mlmc_kgrid_kind kind, uint64_t seed, int64_t first_sample, int64_t M,
                                const double *d_eps, int32_t n_eps, double delta, mlmc_smoother smoother,
                                mlmc_precision prec, double *d_stats, void *d_work, size_t work_bytes,
                                mlmc_stream stream) {
    mlmc_status st = check_level_args(lat, N, coupled, Kf, Kc, prec, n_eps);
    if (st != MLMC_OK) return st;
    if (!(p >= 0.0 && p <= 1.0)) return fail(MLMC_ERR_INVALID_ARG, "level: p = %g", p);
    if (!(delta > 0.0) || !std::isfinite(delta)) return fail(MLMC_ERR_INVALID_ARG, "level: delta = %g", delta);
    if (!valid_kgrid_kind(kind)) return fail(MLMC_ERR_INVALID_ARG, "level: bad k-grid");
    if (smoother != MLMC_SMOOTH_GAUSS && smoother != MLMC_SMOOTH_CUBIC)
        return fail(MLMC_ERR_INVALID_ARG, "level: bad smoother");
    if (M < 0 || first_sample < 0) return fail(MLMC_ERR_INVALID_ARG, "level: negative sample range");
    if (M == 0) return MLMC_OK;
    if (!d_eps || !d_stats) return fail(MLMC_ERR_INVALID_ARG, "level: NULL buffer");
    const bool cpl = coupled != 0;
    const size_t one = level_layout(lat, N, cpl, Kf, Kc, kind, 1, prec, n_eps, nullptr).bytes;
    if (!d_work || work_bytes < one)
        return fail(MLMC_ERR_WORKSPACE, "level: workspace %zu < %zu bytes needed for one sample", work_bytes, one);
    const size_t two = level_layout(lat, N, cpl, Kf, Kc, kind, 2, prec, n_eps, nullptr).bytes;
    const size_t per = two - one, fixed = one - per;
    int64_t mc = (int64_t)((work_bytes - fixed) / per) + 2;  // padding makes the estimate approximate
    if (mc > M) mc = M;
    if (mc < 1) mc = 1;
    while (mc > 1 && level_layout(lat, N, cpl, Kf, Kc, kind, mc, prec, n_eps, nullptr).bytes > work_bytes) --mc;
    const LevelLayout L = level_layout(lat, N, cpl, Kf, Kc, kind, mc, prec, n_eps, static_cast<char *>(d_work));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int G = lat->dev.n_groups, h = N / 2;
    const uint64_t tag = ((uint64_t)lat->dev.lattice_id << 32) | (uint64_t)(uint32_t)N;
    const uint64_t thr = (uint64_t)std::floor(p * 9007199254740992.0);
    const double inv_area_f = 1.0 / ((double)N * N * lat->dev.cell_area);
    const double inv_area_c = cpl ? 1.0 / ((double)h * h * lat->dev.cell_area) : 0.0;
    const int nkf = kgrid_count(kind, Kf), nkc = cpl ? kgrid_count(kind, Kc) : 0;
    const int64_t ldf = (int64_t)lat->dev.n_orb * N * N, ldc = (int64_t)lat->dev.n_orb * h * h;
    // Three streams: the caller's (front) samples, assembles and reduces
    // chunk c (on the two-stage path: stage 1 only); the chase stream chases
    // chunk c's bands on 3/4 of the CUs while the front goes on with chunk
    // c + 1; the back stream runs chunk c's bisection, IDoS and level sums.
    // Matrices (two-stage path), k-grids, sizes, tridiagonals and eigenvalues
    // come in kLevelSets sets used in turn; the front waits until the back
    // has released a set before refilling it.  The sample masks and the
    // stage-1 workspace are the front's alone, the band workspace the chase
    // stream's, the per-sample IDoS the back stream's.
    std::lock_guard<std::mutex> lk(g_back_mu);
    BackStream *bk = nullptr;
    HIP_TRY(back_stream(&bk), "level: back stream");
    hipStream_t sb = bk->s, sc = bk->sc;
    BackStream::LayoutKey key;
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
    // The previous call's front part (masks, stage-1 workspace, the last
    // chunk's matrices) is complete before this call's front starts.
    HIP_TRY(hipStreamWaitEvent(s, bk->ready, 0), "level: wait");
    // Same layout on another stream than the previous call: the caller
    // alternates streams, so the next call is likely to start beside this
    // one's last chunk, which then keeps the chase stream's share of the CUs.
    const bool overlapping = key == bk->last && s != bk->last_stream;
    bk->last_stream = s;
    if (!(key == bk->last)) {
        // Another layout may overlap any of the previous call's buffers: all
        // sets count as released only after everything enqueued so far.
        bk->last = BackStream::LayoutKey{};
        HIP_TRY(hipEventRecord(bk->begin, s), "level: event");
        HIP_TRY(hipStreamWaitEvent(sb, bk->begin, 0), "level: wait");
        for (int q = 0; q < kLevelSets; ++q) HIP_TRY(hipEventRecord(bk->freed[q], sb), "level: event");
        bk->last = key;
        bk->next_set = 0;
    }
    // A call that fails part-way makes the next one take the path above, with
    // the front and chase work it did enqueue covered by `ready` and the back
    // stream.
    struct FailGuard {
        BackStream *bk;
        hipStream_t s;
        bool ok = false;
        ~FailGuard() {
            if (ok) return;
            bk->last = BackStream::LayoutKey{};
            (void)hipEventRecord(bk->chased, bk->sc);
            (void)hipStreamWaitEvent(bk->s, bk->chased, 0);
            (void)hipEventRecord(bk->ready, s);
        }
    } guard{bk, s};
    for (int64_t done = 0; done < M; done += mc) {
        const int64_t ns = (M - done < mc) ? (M - done) : mc;
        const int q = bk->next_set;
        bk->next_set = (q + 1) % kLevelSets;
        HIP_TRY(hipStreamWaitEvent(s, bk->freed[q], 0), "level: wait");
        LAUNCH("kgrid", s, launch_kgrid(kind, Kf, L.kf[q], L.kwf[q], s));
        if (cpl) LAUNCH("kgrid", s, launch_kgrid(kind, Kc, L.kc[q], L.kwc[q], s));
        LAUNCH("sample_vacancies", s, launch_sample_vacancies(lat->dev, N, thr, seed, tag, first_sample + done, ns, L.mask, s));
        bool pend_f = false, pend_c = false, chase_f = false, chase_c = false;
        const EigBuffers bf = L.bf.set(q), bc = L.bc.set(q);
        st = outcome_spectra(lat, N, L.mask, ns, L.kf[q], nkf, prec, L.wf[q], L.nf[q], bf, s, &pend_f, &chase_f);
        if (st != MLMC_OK) return st;
        if (cpl) {
            LAUNCH("partition", s, launch_partition(N, G, L.mask, ns, L.quarters, s));
            st = outcome_spectra(lat, h, L.quarters, ns * 4, L.kc[q], nkc, prec, L.wc[q], L.nc[q], bc, s, &pend_c,
                                 &chase_c);
            if (st != MLMC_OK) return st;
        }
        HIP_TRY(hipEventRecord(bk->ready, s), "level: event");
        HIP_TRY(hipStreamWaitEvent(sb, bk->ready, 0), "level: wait");
        // The last chunk's chase and bisection have nothing left to run
        // beside (unless the calls overlap): they take the whole device (one
        // workgroup per matrix).
        const bool last = !overlapping && done + ns >= M;
        const int64_t chase_blocks = last ? 0 : bk->chase_blocks, bisect_blocks = last ? 0 : bk->bisect_blocks;
        if (chase_f || chase_c) {
            HIP_TRY(hipStreamWaitEvent(sc, bk->ready, 0), "level: wait");
            if (chase_f) {
                st = run_chase(prec, bf.H, ldf, L.nf[q], ns * nkf, bf, sc, chase_blocks);
                if (st != MLMC_OK) return st;
            }
            if (chase_c) {
                st = run_chase(prec, bc.H, ldc, L.nc[q], ns * 4 * nkc, bc, sc, chase_blocks);
                if (st != MLMC_OK) return st;
            }
            HIP_TRY(hipEventRecord(bk->chased, sc), "level: event");
            HIP_TRY(hipStreamWaitEvent(sb, bk->chased, 0), "level: wait");
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
            LAUNCH("idos", sb, launch_idos(L.wc[q], ldc, L.nc[q], ns * 4, nkc, L.kwc[q], inv_area_c, d_eps, n_eps, delta,
                                 (int)smoother, L.Ic, sb));
        }
        LAUNCH("level_stats", sb, launch_level_stats(L.If, cpl ? L.Ic : nullptr, ns, n_eps, d_stats, sb));
        HIP_TRY(hipEventRecord(bk->freed[q], sb), "level: event");
    }
    guard.ok = true;
    HIP_TRY(hipEventRecord(bk->end, sb), "level: event");
    HIP_TRY(hipStreamWaitEvent(s, bk->end, 0), "level: wait");
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

extern "C" {

mlmc_status mlmc_timer_enable(int32_t enable) {
    std::lock_guard<std::mutex> lk(g_timer_mu);
    if (enable) timer_clear_locked();
    g_timing.store(enable != 0);
    return MLMC_OK;
}

mlmc_status mlmc_timer_read(const char *name, double *total_ms, int64_t *launches) {
    if (!name || !total_ms || !launches) return fail(MLMC_ERR_INVALID_ARG, "timer_read: NULL argument");
    std::lock_guard<std::mutex> lk(g_timer_mu);
    double total = 0.0;
    int64_t count = 0;
    for (auto &r : g_timer_recs) {
        if (std::strcmp(r.name, name) != 0) continue;
        HIP_TRY(hipEventSynchronize(r.stop), "timer_read");
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, r.start, r.stop), "timer_read");
        total += ms;
        ++count;
    }
    *total_ms = total;
    *launches = count;
    return MLMC_OK;
}

}  // extern "C"
