// Continuous-batching request server for interior eigen-solves on one GPU.
//
// Requests (matrix, interval, block width, options, seed) are admitted when their
// device footprint fits a byte budget.  Admitted requests of the same matrix and
// filter precision share a pool: three FP64 buffers (plus three in the filter
// precision for the mixed form) of n x cap elements each, handed out in slots: a
// request owning pool columns [c0, c0 + w) owns the contiguous n x w region at
// element offset n * c0 of every buffer (row-major, leading dimension w), so the CSR
// matrix and every request's subspace stay resident and every request's rows are
// contiguous.  Each pool has two host threads, each with its own HIP stream:
//   * the product thread repeats rounds of one grouped Clenshaw product
//     (afsi_clenshaw_step_grouped semantics) for every request that is filtering,
//     whatever product index each one is at - one launch per width for all of them;
//     a request's filtered width is padded up to a width the grouped kernel maps
//     exactly (within its slot; the extra columns are discarded), so slices keep
//     sharing launches after some of their pairs have locked;
//   * the dense thread takes the requests whose filter has finished, one at a time,
//     and runs their dense phases (Cholesky QR, Rayleigh-Ritz, residuals, locking -
//     the steps of Algorithm 4; also the start block's orthonormalisation), so one
//     request's host factorisations never hold up the other slices' products.
// A request moves between the two streams through its own HIP event (recorded on
// the stream that wrote its slot last, waited on by the other).  Requests that
// arrive while others run are admitted as soon as columns and bytes free up;
// independent matrices progress concurrently on their own streams.  A request's
// column arithmetic does not depend on its neighbours, so its results are
// bit-identical alone and in a mix.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <numeric>
#include <thread>
#include <vector>

#include "internal.h"

namespace afsi {
namespace srv {

enum { Q_QUEUED = 0, Q_RUNNING = 1, Q_DONE = 2, Q_FAILED = 3 };
// PH_INIT and PH_DENSE wait for (or run in) the dense thread; PH_FILTER is the product
// thread's; PH_GONE: finished, to be dropped by the product thread.
enum { PH_INIT = 0, PH_FILTER = 1, PH_DENSE = 2, PH_GONE = 3 };

struct Pool;

// Dense threads per pool: the dense phases of that many requests run concurrently,
// each on its own stream (they are host-latency bound: small factorisations between
// device steps).
constexpr int kDenseWorkers = 2;

struct Request {
    int64_t id = 0;
    afsi_matrix_t A = nullptr;
    double a = 0, b = 0;
    int64_t p = 0;
    afsi_options opts{};
    uint64_t seed = 0;
    int dt = AFSI_R64, fdt = AFSI_R64;
    int state = Q_QUEUED, status = AFSI_OK;
    std::string error;
    double t_submit = 0, t_admit = 0, t_done = 0;
    std::vector<double> lam, res;
    void *evecs = nullptr;  // n x p, ld = p, FP64 domain dtype
    int64_t n_lock = 0;
    int iterations = 0, converged = 0;
    int64_t spmv = 0;
    double avg_degree = 0;
    size_t evec_bytes = 0;
};

struct Session {
    Request *r = nullptr;
    int64_t col0 = 0, cap = 0, p_act = 0;
    std::vector<double> coeffs;
    double l1 = 0, l2 = 0, tau_abs = 0;
    int k_cur = 1, step = 0, phase = PH_INIT;
    int64_t n_check_prev = 0;
    std::vector<int> degrees;
    hipEvent_t ev = nullptr;    // last write to the slot, on the stream that made it
    bool ev_recorded = false;   // ev holds a record to wait for
    bool in_dense = false;      // owned by the dense thread (queued or running)
};

struct Server;

struct Pool {
    Server *S = nullptr;
    afsi_matrix_t A = nullptr;
    int dt = AFSI_R64, fdt = AFSI_R64;
    int64_t n = 0, cap = 0, E = 1;
    void *B[3] = {nullptr, nullptr, nullptr};  // FP64: active block, filter output / Q, work / AV
    void *F[3] = {nullptr, nullptr, nullptr};  // filter precision (mixed form only)
    hipStream_t stream = nullptr;                  // products (product thread)
    hipStream_t dstream[kDenseWorkers] = {};       // dense phases, one per dense thread
    std::thread dense[kDenseWorkers];
    std::deque<Session *> dense_q;  // sessions handed to the dense thread (under S->mu)
    std::deque<Session *> back_q;   // sessions it has handed back (under S->mu)
    bool dense_stop = false;
    int64_t in_dense = 0;
    std::vector<uint8_t> used;  // per column
    std::list<Session> sessions;
    std::deque<Session> incoming;
    size_t bytes = 0;
    size_t blk = 0, fblk = 0;  // bytes of each FP64 / filter-precision buffer
    bool mixed() const { return fdt != dt; }
};

// Device memory of a server: chunks obtained with hipMalloc as needed and returned only
// when the server is destroyed; pool buffers and eigenvector blocks are carved out of
// them first-fit and given back (with coalescing) when their request or pool ends.
// hipMalloc / hipFree of multi-GB buffers during a stream took seconds at times and
// hipFree waits for the whole device, so the stream itself never calls them.
struct Arena {
    static constexpr size_t kAlign = 4096;
    static constexpr size_t kChunkMin = size_t(8) << 30;
    struct Chunk {
        char *base = nullptr;
        size_t size = 0;
        std::map<size_t, size_t> free;  // offset -> length, disjoint and not adjacent
    };
    std::vector<Chunk> chunks;

    // caller holds the server lock; throws on a failed hipMalloc
    void *alloc(size_t bytes) {
        bytes = std::max<size_t>((bytes + kAlign - 1) / kAlign * kAlign, kAlign);
        for (auto &c : chunks)
            for (auto it = c.free.begin(); it != c.free.end(); ++it)
                if (it->second >= bytes) {
                    const size_t off = it->first, len = it->second;
                    c.free.erase(it);
                    if (len > bytes) c.free[off + bytes] = len - bytes;
                    return c.base + off;
                }
        Chunk c;
        c.size = std::max(bytes, kChunkMin);
        void *p = nullptr;
        if (hipMalloc(&p, c.size) != hipSuccess) {
            (void)hipGetLastError();
            c.size = bytes;  // the rest of the device may still hold exactly this block
            AFSI_HIP(hipMalloc(&p, c.size));
        }
        c.base = static_cast<char *>(p);
        if (c.size > bytes) c.free[bytes] = c.size - bytes;
        chunks.push_back(std::move(c));
        return p;
    }
    // caller holds the server lock, and no work that uses the block is still queued
    void release(void *p, size_t bytes) {
        if (!p) return;
        bytes = std::max<size_t>((bytes + kAlign - 1) / kAlign * kAlign, kAlign);
        for (auto &c : chunks) {
            char *q = static_cast<char *>(p);
            if (q < c.base || q >= c.base + c.size) continue;
            size_t off = (size_t)(q - c.base), len = bytes;
            auto next = c.free.lower_bound(off);
            if (next != c.free.end() && off + len == next->first) {
                len += next->second;
                next = c.free.erase(next);
            }
            if (next != c.free.begin()) {
                auto prev = std::prev(next);
                if (prev->first + prev->second == off) {
                    off = prev->first;
                    len += prev->second;
                    c.free.erase(prev);
                }
            }
            c.free[off] = len;
            return;
        }
    }
    void destroy() {
        for (auto &c : chunks) (void)hipFree(c.base);
        chunks.clear();
    }
};

struct Server {
    int device = 0;
    int64_t budget = 0, in_use = 0;
    Arena arena;
    std::mutex mu;
    std::condition_variable cv;     // request completions / thread exits
    std::deque<Request *> queue;
    std::map<int64_t, std::unique_ptr<Request>> reqs;
    std::map<std::pair<afsi_matrix_t, int>, Pool *> pools;
    std::map<afsi_matrix_t, int64_t> pool_cols;
    std::deque<int64_t> finished;
    int64_t next_id = 1, n_done = 0;
    int live_threads = 0;
    bool stopping = false;
    int64_t launches = 0, launch_groups = 0;
    int64_t kernel_launches = 0, kernel_slices = 0;  // grouped kernel launches / slices they took
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

int64_t col_align(int dt, int fdt) {
    return std::max<int64_t>(16 / elem_bytes(dt), 16 / elem_bytes(fdt));
}

size_t pool_bytes(int64_t n, int64_t cap, int dt, int fdt) {
    size_t b = 3 * (size_t)n * cap * elem_bytes(dt);
    if (fdt != dt) b += 3 * (size_t)n * cap * elem_bytes(fdt);
    return b;
}

int64_t find_run(const std::vector<uint8_t> &used, int64_t need, int64_t E) {
    const int64_t cap = (int64_t)used.size();
    for (int64_t c = 0; c + need <= cap; c += E) {
        bool ok = true;
        for (int64_t j = c; j < c + need; ++j)
            if (used[j]) {
                ok = false;
                break;
            }
        if (ok) return c;
    }
    return -1;
}

void pool_thread(Pool *P);

// A queued request that cannot be started (caller holds S->mu; the caller removes
// it from the queue).
void fail_queued(Server *S, Request *r, int status, const char *msg) {
    r->state = Q_FAILED;
    r->status = status;
    r->error = msg;
    r->t_done = S->now();
    S->finished.push_back(r->id);
    ++S->n_done;
}

// Admit every queued request that fits (caller holds S->mu).
void try_admit(Server *S) {
    for (auto it = S->queue.begin(); it != S->queue.end();) {
        Request *r = *it;
        const auto key = std::make_pair(r->A, r->fdt);
        const int64_t E = col_align(r->dt, r->fdt);
        const int64_t need = round_up(r->p, E);
        Pool *P = nullptr;
        auto pit = S->pools.find(key);
        int64_t col0 = -1;
        size_t new_pool = 0;
        if (pit != S->pools.end()) {
            P = pit->second;
            col0 = find_run(P->used, need, E);
            if (col0 < 0) {
                ++it;
                continue;
            }
        } else {
            int64_t cap = need;
            auto h = S->pool_cols.find(r->A);
            if (h != S->pool_cols.end()) cap = std::max(cap, round_up(h->second, E));
            new_pool = pool_bytes(r->A->n, cap, r->dt, r->fdt);
            if (S->in_use + (int64_t)(new_pool + r->evec_bytes) > S->budget) {
                ++it;
                continue;
            }
            std::unique_ptr<Pool> np(new Pool());
            np->S = S;
            np->A = r->A;
            np->dt = r->dt;
            np->fdt = r->fdt;
            np->n = r->A->n;
            np->cap = cap;
            np->E = E;
            np->used.assign(cap, 0);
            np->blk = (size_t)np->n * cap * elem_bytes(r->dt);
            np->fblk = np->mixed() ? (size_t)np->n * cap * elem_bytes(r->fdt) : 0;
            try {
                DeviceGuard dg(S->device);
                for (auto &b : np->B) b = S->arena.alloc(np->blk);
                if (np->mixed())
                    for (auto &b : np->F) b = S->arena.alloc(np->fblk);
                AFSI_HIP(hipStreamCreateWithFlags(&np->stream, hipStreamNonBlocking));
                for (auto &d : np->dstream) AFSI_HIP(hipStreamCreateWithFlags(&d, hipStreamNonBlocking));
            } catch (...) {
                for (auto &b : np->B) S->arena.release(b, np->blk), b = nullptr;
                for (auto &b : np->F) S->arena.release(b, np->fblk), b = nullptr;
                if (np->stream) (void)hipStreamDestroy(np->stream);
                for (auto d : np->dstream)
                    if (d) (void)hipStreamDestroy(d);
                fail_queued(S, r, AFSI_E_NOMEM, "device allocation of the request's pool failed");
                it = S->queue.erase(it);
                continue;
            }
            np->bytes = new_pool;
            S->in_use += (int64_t)new_pool;
            P = np.release();
            S->pools[key] = P;
            ++S->live_threads;
            std::thread(pool_thread, P).detach();
            col0 = 0;
        }
        if (S->in_use + (int64_t)r->evec_bytes > S->budget) {
            ++it;
            continue;
        }
        try {
            DeviceGuard dg(S->device);
            r->evecs = S->arena.alloc(r->evec_bytes);
        } catch (...) {
            r->evecs = nullptr;
            fail_queued(S, r, AFSI_E_NOMEM, "device allocation of the eigenvector block failed");
            it = S->queue.erase(it);
            continue;
        }
        S->in_use += (int64_t)r->evec_bytes;
        for (int64_t j = col0; j < col0 + need; ++j) P->used[j] = 1;
        Session s;
        s.r = r;
        s.col0 = col0;
        s.cap = need;
        s.p_act = r->p;
        r->state = Q_RUNNING;
        r->t_admit = S->now();
        P->incoming.push_back(std::move(s));
        it = S->queue.erase(it);
    }
    S->cv.notify_all();
}

void *col_ptr(void *base, int64_t col, int dt) {
    return (char *)base + (size_t)col * elem_bytes(dt);
}

// A session's n x s.cap region of one pool buffer (leading dimension s.cap).
void *slot_ptr(const Pool *P, void *base, const Session &s, int dt) {
    return (char *)base + (size_t)P->n * s.col0 * elem_bytes(dt);
}

void finish(Pool *P, Session &s, int status, const std::string &err) {
    Server *S = P->S;
    Request *r = s.r;
    std::lock_guard<std::mutex> lk(S->mu);
    r->status = status;
    r->error = err;
    r->state = (status == AFSI_OK || status == AFSI_E_NOCONV) ? Q_DONE : Q_FAILED;
    r->converged = status == AFSI_OK;
    r->avg_degree = s.degrees.empty()
                        ? 0.0
                        : std::accumulate(s.degrees.begin(), s.degrees.end(), 0.0) / s.degrees.size();
    r->t_done = S->now();
    for (int64_t j = s.col0; j < s.col0 + s.cap; ++j) P->used[j] = 0;
    S->finished.push_back(r->id);
    ++S->n_done;
    S->cv.notify_all();
}

// Start block from the request's seed, orthonormalised (Algorithm 4, initialisation).
void init_session(Pool *P, Session &s, hipStream_t st) {
    Request *r = s.r;
    const int comp = is_complex(P->dt) ? 2 : 1;
    void *B0 = slot_ptr(P, P->B[0], s, P->dt);
    launch_fill_normal((double *)B0, P->n, r->p, s.cap, comp, r->seed, st);
    orthonormalize_dev(P->dt, B0, slot_ptr(P, P->B[1], s, P->dt), P->n, r->p, s.cap, st,
                       nullptr);
    s.coeffs.resize(r->opts.kmax + 1);
    filter_coefficients(r->A->lmin, r->A->lmax, r->a, r->b, r->opts.kmax, r->opts.damping,
                        r->opts.m_exp, s.coeffs.data());
    const double w = r->A->lmax - r->A->lmin;
    s.l1 = 2.0 / w;
    s.l2 = -(r->A->lmax + r->A->lmin) / w;
    s.tau_abs = r->opts.tau_c * std::max(std::fabs(r->A->lmin), std::fabs(r->A->lmax));
    s.k_cur = r->opts.kmax;
    if (r->opts.k_init > 0) {
        s.k_cur = std::min(r->opts.k_init, r->opts.kmax);
    } else if (r->opts.adaptive) {
        const double ta = std::min(1.0, std::max(-1.0, (2 * r->a - r->A->lmax - r->A->lmin) / w));
        const double tb = std::min(1.0, std::max(-1.0, (2 * r->b - r->A->lmax - r->A->lmin) / w));
        s.k_cur = std::max(1, std::min((int)std::ceil(r->opts.C / (std::acos(ta) - std::acos(tb))) - 1,
                                       r->opts.kmax));
    }
}

void start_filter(Pool *P, Session &s, hipStream_t st) {
    s.phase = PH_FILTER;
    s.step = 0;
    if (P->mixed()) {
        afsi_block src{slot_ptr(P, P->B[0], s, P->dt), P->n, s.p_act, s.cap, P->dt};
        afsi_block dst{slot_ptr(P, P->F[0], s, P->fdt), P->n, s.p_act, s.cap, P->fdt};
        launch_convert(src, dst, st);
    }
}

enum { DP_CONTINUE = 0, DP_CONVERGED = 1, DP_LIMIT = 2 };

// Progress counters that afsi_server_info reads while the request runs: updated
// under the server lock (the pool thread is their only writer).
void publish(Pool *P, Request *r, int iterations, int64_t spmv, int64_t locked) {
    std::lock_guard<std::mutex> lk(P->S->mu);
    r->iterations += iterations;
    r->spmv += spmv;
    r->n_lock += locked;
}

// One pass of the dense steps after a filter; says whether the request goes on.
int dense_phase(Pool *P, Session &s, hipStream_t st) {
    Request *r = s.r;
    const int dt = P->dt;
    const int64_t n = P->n, ld = s.cap, pa = s.p_act;
    const int outi = 1 + (s.k_cur - 1) % 2;  // product output lands in P[(k-1) % 2]
    void *q, *w;
    if (P->mixed()) {
        afsi_block src{slot_ptr(P, P->F[outi], s, P->fdt), n, pa, ld, P->fdt};
        afsi_block dst{slot_ptr(P, P->B[1], s, dt), n, pa, ld, dt};
        launch_convert(src, dst, st);
        q = slot_ptr(P, P->B[1], s, dt);
        w = slot_ptr(P, P->B[2], s, dt);
    } else {
        q = slot_ptr(P, P->B[outi], s, dt);
        w = slot_ptr(P, P->B[3 - outi], s, dt);
    }
    void *v = slot_ptr(P, P->B[0], s, dt);
    s.degrees.push_back(s.k_cur);
    publish(P, r, 1, (int64_t)s.k_cur * pa, 0);
    if (r->n_lock > 0) project_out_dev(dt, r->evecs, r->p, r->n_lock, q, ld, n, pa, st);
    double maxn2 = 0.0;
    std::vector<double> ritz(pa), res(pa);
    orthonormalize_rr_dev(r->A, dt, q, w, v, w, n, pa, ld, ritz.data(), st, &maxn2, nullptr);
    if (r->opts.damping != AFSI_DAMP_NONE && maxn2 > 16.0)
        AFSI_FAIL(AFSI_E_BOUNDS, "filtered block grew by %.3g: spectral bounds do not enclose A",
                  std::sqrt(maxn2));
    publish(P, r, 0, pa, 0);
    std::vector<uint8_t> I(pa), lock(pa);
    int64_t e = 0;
    for (int64_t j = 0; j < pa; ++j) {
        I[j] = ritz[j] >= r->a && ritz[j] <= r->b;
        e += I[j];
    }
    if (e > 0) {
        if (r->opts.adaptive)
            s.k_cur = select_degree(ritz.data(), pa, e, s.coeffs.data(), r->opts.kmax, s.l1, s.l2,
                                    r->opts.tau_a);
        residual_norms_host(dt, v, ld, w, ld, ritz.data(), n, pa, res.data(), st);
        int done = 0;
        lock_select(ritz.data(), pa, res.data(), I.data(), r->a, r->b, s.tau_abs, r->n_lock,
                    &s.n_check_prev, lock.data(), &done);
        std::vector<int32_t> lk, keep;
        for (int64_t j = 0; j < pa; ++j) (lock[j] ? lk : keep).push_back((int32_t)j);
        if (!lk.empty()) {
            AFSI_REQUIRE(r->n_lock + (int64_t)lk.size() <= r->p, "locked more pairs than columns");
            for (auto j : lk) {
                r->lam.push_back(ritz[j]);
                r->res.push_back(res[j]);
            }
            gather_cols(dt, v, n, ld, lk.data(), (int64_t)lk.size(), col_ptr(r->evecs, r->n_lock, dt),
                        r->p, st);
            if (!keep.empty()) {
                gather_cols(dt, v, n, ld, keep.data(), (int64_t)keep.size(), w, ld, st);
                const int eb = elem_bytes(dt);
                AFSI_HIP(hipMemcpy2DAsync(v, ld * eb, w, ld * eb, keep.size() * eb, n,
                                          hipMemcpyDeviceToDevice, st));
            }
            publish(P, r, 0, 0, (int64_t)lk.size());
            s.p_act -= (int64_t)lk.size();
        }
        if (done) return DP_CONVERGED;
    }
    if (r->iterations >= r->opts.max_iter) return DP_LIMIT;
    start_filter(P, s, st);
    return DP_CONTINUE;
}

void sort_results(Pool *P, const Session &s, Request *r, hipStream_t st) {
    if (r->n_lock < 2) return;
    std::vector<int32_t> order(r->n_lock);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return r->lam[x] < r->lam[y]; });
    std::vector<double> lam(r->n_lock), res(r->n_lock);
    for (int64_t t = 0; t < r->n_lock; ++t) lam[t] = r->lam[order[t]], res[t] = r->res[order[t]];
    r->lam = lam;
    r->res = res;
    // permute the eigenvector columns through the request's slot of the pool's work
    // buffer (n x s.cap, free once the dense phase is over; n_lock <= p <= s.cap)
    const int dt = P->dt, eb = elem_bytes(dt);
    void *tmp = slot_ptr(P, P->B[2], s, dt);
    gather_cols(dt, r->evecs, P->n, r->p, order.data(), r->n_lock, tmp, s.cap, st);
    AFSI_HIP(hipMemcpy2DAsync(r->evecs, r->p * eb, tmp, s.cap * eb, r->n_lock * eb, P->n,
                              hipMemcpyDeviceToDevice, st));
    AFSI_HIP(hipStreamSynchronize(st));
}

// Stream of a pool that has left S->pools (so no request can be admitted to it): wait
// for its work, then destroy it.  Called without S->mu; afterwards, under the lock, the
// caller gives the pool's buffers back to the arena.
void retire_pool_stream(Pool *P) {
    (void)hipStreamSynchronize(P->stream);
    (void)hipStreamDestroy(P->stream);
    for (hipStream_t st : P->dstream) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
}

// Filtered width of a session: its active columns rounded up to whole 16-byte vectors,
// then up to the nearest width the grouped kernel maps exactly if that fits the slot.
int64_t filter_width(const Pool *P, const Session &s) {
    const int64_t nc = round_up(s.p_act, P->E);
    const int eb = elem_bytes(P->fdt);
    const int64_t w16 = grouped_width_at_least(nc * eb / 16);
    if (w16 > 0 && w16 * 16 / eb <= s.cap) return w16 * 16 / eb;
    return nc;
}

// A dense thread of a pool: start blocks (PH_INIT) and the dense phases after each
// filter (PH_DENSE), one session at a time, on the thread's own stream.
void dense_thread(Pool *P, int worker) {
    Server *S = P->S;
    (void)hipSetDevice(S->device);
    hipStream_t st = P->dstream[worker];
    for (;;) {
        Session *sp = nullptr;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv.wait(lk, [&] { return !P->dense_q.empty() || P->dense_stop; });
            if (P->dense_q.empty()) return;  // dense_stop and nothing left
            sp = P->dense_q.front();
            P->dense_q.pop_front();
            if (S->stopping) {  // hand it back untouched: the product thread fails it
                P->back_q.push_back(sp);
                S->cv.notify_all();
                continue;
            }
        }
        Session &s = *sp;
        try {
            if (s.ev_recorded) AFSI_HIP(hipStreamWaitEvent(st, s.ev, 0));
            if (s.phase == PH_INIT) {
                init_session(P, s, st);
                start_filter(P, s, st);
            } else {
                const int outcome = dense_phase(P, s, st);
                if (outcome != DP_CONTINUE) {
                    sort_results(P, s, s.r, st);
                    finish(P, s, outcome == DP_CONVERGED ? AFSI_OK : AFSI_E_NOCONV, "");
                    s.phase = PH_GONE;
                }
            }
            if (s.phase != PH_GONE) {
                AFSI_HIP(hipEventRecord(s.ev, st));
                s.ev_recorded = true;
            }
        } catch (const Error &e) {
            // nothing of this request may still run when its columns are given back
            if (s.ev_recorded) (void)hipEventSynchronize(s.ev);
            (void)hipStreamSynchronize(st);
            finish(P, s, e.status, afsi_last_error());
            s.phase = PH_GONE;
        } catch (const std::exception &e) {
            if (s.ev_recorded) (void)hipEventSynchronize(s.ev);
            (void)hipStreamSynchronize(st);
            finish(P, s, AFSI_E_NOMEM, e.what());
            s.phase = PH_GONE;
        }
        std::lock_guard<std::mutex> lk(S->mu);
        P->back_q.push_back(sp);
        S->cv.notify_all();
    }
}

// Launches the product thread keeps queued ahead of the device: it waits for launch
// i - kAhead before issuing launch i, so requests that arrive or come back from their
// dense phase join the next rounds instead of queueing behind a whole filter.
constexpr int kAhead = 3;

void pool_thread(Pool *P) {
    Server *S = P->S;
    (void)hipSetDevice(S->device);
    hipEvent_t ahead[kAhead] = {};
    for (auto &e : ahead)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            e = nullptr;
        }
    int64_t rounds = 0;
    for (int w = 0; w < kDenseWorkers; ++w) P->dense[w] = std::thread(dense_thread, P, w);
    std::vector<afsi_slice_blocks> groups;
    std::vector<Session *> filt;
    std::vector<Session *> fresh, back;
    for (;;) {
        fresh.clear();
        back.clear();
        {
            std::unique_lock<std::mutex> lk(S->mu);
            for (;;) {
                while (!P->incoming.empty()) {
                    P->sessions.push_back(std::move(P->incoming.front()));
                    P->incoming.pop_front();
                    fresh.push_back(&P->sessions.back());
                }
                for (Session *sp : P->back_q) {
                    sp->in_dense = false;
                    back.push_back(sp);
                }
                P->in_dense -= (int64_t)P->back_q.size();
                P->back_q.clear();
                bool filtering = false;
                for (auto &x : P->sessions) filtering |= !x.in_dense && x.phase == PH_FILTER;
                const bool idle = P->sessions.empty() && P->in_dense == 0;
                if (filtering || !fresh.empty() || !back.empty() || idle || S->stopping) break;
                S->cv.wait(lk);
            }
            const bool gone = std::all_of(P->sessions.begin(), P->sessions.end(),
                                          [](const Session &x) { return x.phase == PH_GONE; });
            if ((gone && P->in_dense == 0) || S->stopping) {
                // leave the pool table first, under the lock that admission holds: no
                // request can be admitted into this pool from here on
                S->pools.erase(std::make_pair(P->A, P->fdt));
                P->dense_stop = true;
                S->cv.notify_all();
                lk.unlock();
                for (auto &th : P->dense) th.join();  // they return once the queue is empty
                lk.lock();
                for (Session *sp : P->back_q) sp->in_dense = false;
                P->back_q.clear();
                P->in_dense = 0;
                for (auto &x : P->sessions) {
                    if (x.phase == PH_GONE) continue;
                    x.r->state = Q_FAILED;
                    x.r->status = AFSI_E_INVALID;
                    x.r->error = "server stopped";
                }
                lk.unlock();
                retire_pool_stream(P);
                for (auto &x : P->sessions)
                    if (x.ev) (void)hipEventDestroy(x.ev);
                for (auto e : ahead)
                    if (e) (void)hipEventDestroy(e);
                lk.lock();
                for (auto b : P->B) S->arena.release(b, P->blk);
                for (auto b : P->F) S->arena.release(b, P->fblk);
                S->in_use -= (int64_t)P->bytes;
                --S->live_threads;
                try_admit(S);
                S->cv.notify_all();
                delete P;
                return;
            }
        }
        // finished sessions leave; new ones go to the dense thread for their start block
        P->sessions.remove_if([](Session &x) {
            if (x.phase != PH_GONE || x.in_dense) return false;
            if (x.ev) (void)hipEventDestroy(x.ev);
            return true;
        });
        std::vector<Session *> to_dense;
        for (Session *sp : fresh) {
            if (hipEventCreateWithFlags(&sp->ev, hipEventDisableTiming) != hipSuccess) {
                (void)hipGetLastError();
                sp->ev = nullptr;
                finish(P, *sp, AFSI_E_HIP, "hipEventCreate failed");
                sp->phase = PH_GONE;
                continue;
            }
            to_dense.push_back(sp);
        }
        // sessions back from the dense thread with a filter to run: the product stream
        // waits for their dense work
        for (Session *sp : back)
            if (sp->phase == PH_FILTER && sp->ev_recorded &&
                hipStreamWaitEvent(P->stream, sp->ev, 0) != hipSuccess) {
                (void)hipGetLastError();
                for (hipStream_t d : P->dstream) (void)hipStreamSynchronize(d);
            }
        filt.clear();
        groups.clear();
        for (auto &x : P->sessions)
            if (!x.in_dense && x.phase == PH_FILTER) {
                afsi_slice_blocks g{};
                step_params(x.coeffs.data(), x.k_cur, x.step, x.l1, x.l2, &g.step);
                g.step.col0 = 0;
                g.step.ncols = filter_width(P, x);
                g.step.active = 1;
                void **buf = P->mixed() ? P->F : P->B;
                g.X = slot_ptr(P, buf[0], x, P->fdt);
                g.P0 = slot_ptr(P, buf[1], x, P->fdt);
                g.P1 = slot_ptr(P, buf[2], x, P->fdt);
                g.ld = x.cap;
                groups.push_back(g);
                filt.push_back(&x);
            }
        try {
            if (!groups.empty()) {
                hipEvent_t &slot = ahead[rounds % kAhead];
                if (rounds >= kAhead && slot) AFSI_HIP(hipEventSynchronize(slot));
                int klaunch = 0;
                const int taken = grouped_step(P->A, (int)groups.size(), groups.data(), P->fdt,
                                               P->stream, &klaunch);
                if (slot) AFSI_HIP(hipEventRecord(slot, P->stream));
                ++rounds;
                std::lock_guard<std::mutex> lk(S->mu);
                ++S->launches;
                S->launch_groups += (int64_t)groups.size();
                S->kernel_launches += klaunch;
                S->kernel_slices += taken;
            }
            for (auto *x : filt)
                if (++x->step == x->k_cur) {
                    x->phase = PH_DENSE;
                    AFSI_HIP(hipEventRecord(x->ev, P->stream));
                    x->ev_recorded = true;
                    to_dense.push_back(x);
                }
        } catch (const Error &e) {
            // none of filt has reached the dense thread yet
            const std::string msg = afsi_last_error();
            (void)hipStreamSynchronize(P->stream);
            for (auto *x : filt) x->phase = PH_GONE, finish(P, *x, e.status, msg);
            to_dense.erase(std::remove_if(to_dense.begin(), to_dense.end(),
                                          [](Session *x) { return x->phase == PH_GONE; }),
                           to_dense.end());
        } catch (const std::exception &e) {
            (void)hipStreamSynchronize(P->stream);
            for (auto *x : filt) x->phase = PH_GONE, finish(P, *x, AFSI_E_NOMEM, e.what());
            to_dense.erase(std::remove_if(to_dense.begin(), to_dense.end(),
                                          [](Session *x) { return x->phase == PH_GONE; }),
                           to_dense.end());
        }
        if (!to_dense.empty()) {
            std::lock_guard<std::mutex> lk(S->mu);
            for (Session *sp : to_dense) {
                sp->in_dense = true;
                P->dense_q.push_back(sp);
            }
            P->in_dense += (int64_t)to_dense.size();
            S->cv.notify_all();
        }
    }
}

}  // namespace srv
}  // namespace afsi

struct afsi_server_s : afsi::srv::Server {};

using namespace afsi;
using namespace afsi::srv;

extern "C" {

int afsi_server_create(int device, int64_t hbm_budget_bytes, afsi_server_t *out) {
    return guarded([&] {
        AFSI_REQUIRE(out != nullptr && hbm_budget_bytes > 0, "bad argument");
        DeviceGuard dg(device);
        auto *S = new afsi_server_s();
        S->device = device;
        S->budget = hbm_budget_bytes;
        *out = S;
    });
}

int afsi_server_destroy(afsi_server_t S) {
    return guarded([&] {
        if (!S) return;
        std::unique_lock<std::mutex> lk(S->mu);
        S->stopping = true;
        for (Request *r : S->queue) r->state = Q_FAILED, r->error = "server stopped";
        S->queue.clear();
        S->cv.wait(lk, [&] { return S->live_threads == 0; });
        DeviceGuard dg(S->device);
        (void)hipDeviceSynchronize();
        S->arena.destroy();  // every pool and eigenvector block lives in it
        lk.unlock();
        delete S;
    });
}

int afsi_server_set_pool_columns(afsi_server_t S, afsi_matrix_t A, int64_t cols) {
    return guarded([&] {
        AFSI_REQUIRE(S && A && cols > 0, "bad argument");
        std::lock_guard<std::mutex> lk(S->mu);
        S->pool_cols[A] = cols;
    });
}

int afsi_server_submit(afsi_server_t S, afsi_matrix_t A, double a, double b, int64_t p,
                       const afsi_options *opts, uint64_t seed, int64_t *id) {
    return guarded([&] {
        AFSI_REQUIRE(S && A && opts && id, "NULL argument");
        AFSI_REQUIRE(A->device == S->device, "matrix lives on another device");
        AFSI_REQUIRE(A->has_bounds, "spectral bounds are not set on this matrix");
        AFSI_REQUIRE(b > a && p >= 1 && p <= A->n, "need a < b and 1 <= p <= n");
        AFSI_REQUIRE(opts->kmax >= 1 && opts->max_iter >= 1, "kmax and max_iter must be >= 1");
        const int dt = A->dtype;
        const int fdt = opts->filter_dtype;
        AFSI_REQUIRE(fdt >= AFSI_R64 && fdt <= AFSI_C64 && is_complex(fdt) == is_complex(dt),
                     "filter dtype must match the matrix domain");
        std::unique_ptr<Request> r(new Request());
        r->A = A;
        r->a = a;
        r->b = b;
        r->p = p;
        r->opts = *opts;
        r->seed = seed;
        r->dt = dt;
        r->fdt = fdt;
        r->evec_bytes = (size_t)A->n * p * elem_bytes(dt);
        const size_t alone = pool_bytes(A->n, round_up(p, col_align(dt, fdt)), dt, fdt) + r->evec_bytes;
        if ((int64_t)alone > S->budget)
            AFSI_FAIL(AFSI_E_BUSY, "request needs %zu bytes, the budget is %lld", alone,
                      (long long)S->budget);
        std::lock_guard<std::mutex> lk(S->mu);
        AFSI_REQUIRE(!S->stopping, "server is stopping");
        r->id = S->next_id++;
        r->t_submit = S->now();
        *id = r->id;
        S->queue.push_back(r.get());
        S->reqs[r->id] = std::move(r);
        try_admit(S);
    });
}

static void fill_info(const Request *r, afsi_request_info *info) {
    info->state = r->state;
    info->status = r->status;
    info->count = r->n_lock;
    info->iterations = r->iterations;
    info->converged = r->converged;
    info->spmv = r->spmv;
    info->avg_degree = r->avg_degree;
    info->t_submit = r->t_submit;
    info->t_admit = r->t_admit;
    info->t_done = r->t_done;
}

int afsi_server_info(afsi_server_t S, int64_t id, afsi_request_info *info) {
    return guarded([&] {
        AFSI_REQUIRE(S && info, "NULL argument");
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->reqs.find(id);
        AFSI_REQUIRE(it != S->reqs.end(), "unknown request %lld", (long long)id);
        fill_info(it->second.get(), info);
    });
}

int afsi_server_wait(afsi_server_t S, int64_t id, double timeout_s, afsi_request_info *info) {
    return guarded([&] {
        AFSI_REQUIRE(S && info, "NULL argument");
        std::unique_lock<std::mutex> lk(S->mu);
        auto it = S->reqs.find(id);
        AFSI_REQUIRE(it != S->reqs.end(), "unknown request %lld", (long long)id);
        Request *r = it->second.get();
        S->cv.wait_for(lk, std::chrono::duration<double>(timeout_s),
                       [&] { return r->state >= Q_DONE; });
        fill_info(r, info);
    });
}

int afsi_server_wait_any(afsi_server_t S, double timeout_s, int64_t *id) {
    return guarded([&] {
        AFSI_REQUIRE(S && id, "NULL argument");
        std::unique_lock<std::mutex> lk(S->mu);
        S->cv.wait_for(lk, std::chrono::duration<double>(timeout_s),
                       [&] { return !S->finished.empty(); });
        if (S->finished.empty()) {
            *id = -1;
        } else {
            *id = S->finished.front();
            S->finished.pop_front();
        }
    });
}

int afsi_server_fetch(afsi_server_t S, int64_t id, double *eigenvalues, double *residuals,
                      int64_t capacity, afsi_block *evecs, void *stream) {
    return guarded([&] {
        AFSI_REQUIRE(S, "NULL server");
        std::unique_ptr<Request> r;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            auto it = S->reqs.find(id);
            AFSI_REQUIRE(it != S->reqs.end(), "unknown request %lld", (long long)id);
            AFSI_REQUIRE(it->second->state >= Q_DONE, "request %lld has not finished", (long long)id);
            AFSI_REQUIRE(capacity >= it->second->n_lock, "capacity %lld < %lld eigenpairs",
                         (long long)capacity, (long long)it->second->n_lock);
            if (evecs) {
                AFSI_REQUIRE(evecs->dtype == it->second->dt && evecs->rows == it->second->A->n &&
                                 evecs->cols >= it->second->n_lock,
                             "evecs must be n x count of the matrix's FP64 dtype");
            }
            r = std::move(it->second);
            S->reqs.erase(it);
        }
        const int64_t cnt = r->n_lock;
        if (cnt) {
            if (eigenvalues) std::memcpy(eigenvalues, r->lam.data(), sizeof(double) * cnt);
            if (residuals) std::memcpy(residuals, r->res.data(), sizeof(double) * cnt);
        }
        DeviceGuard dg(S->device);
        if (evecs && cnt && r->A->n) {
            const int eb = elem_bytes(r->dt);
            hipStream_t s = reinterpret_cast<hipStream_t>(stream);
            AFSI_HIP(hipMemcpy2DAsync(evecs->ptr, evecs->ld * eb, r->evecs, r->p * eb, cnt * eb,
                                      r->A->n, hipMemcpyDeviceToDevice, s));
            AFSI_HIP(hipStreamSynchronize(s));
        }
        // the pool thread synchronised its stream after the last write to evecs, and the
        // copy above is complete: the block can go back to the arena
        std::lock_guard<std::mutex> lk(S->mu);
        if (r->evecs) {
            S->arena.release(r->evecs, r->evec_bytes);
            r->evecs = nullptr;
            S->in_use -= (int64_t)r->evec_bytes;
        }
        try_admit(S);
    });
}

int afsi_server_get_stats(afsi_server_t S, afsi_server_stats *st) {
    return guarded([&] {
        AFSI_REQUIRE(S && st, "NULL argument");
        std::lock_guard<std::mutex> lk(S->mu);
        st->bytes_in_use = S->in_use;
        st->budget = S->budget;
        st->queued = (int64_t)S->queue.size();
        int64_t running = 0;
        for (auto &kv : S->reqs) running += kv.second->state == Q_RUNNING;
        st->running = running;
        st->done = S->n_done;
        st->pools = (int64_t)S->pools.size();
        st->batched_launches = S->launches;
        st->batched_groups = S->launch_groups;
        st->kernel_launches = S->kernel_launches;
        st->kernel_slices = S->kernel_slices;
        st->now = S->now();
    });
}

}  // extern "C"
