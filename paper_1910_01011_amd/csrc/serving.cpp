// Continuous batching of operator applies across problems (serving).
//
// Requests are solved side by side, each by its own host thread on its own
// stream (its Krylov work, right-hand sides and preconditioner stay there).
// A problem attached to a bem_batch hands every operator apply of its solves to
// the batch's dispatcher instead of launching it.  The dispatcher gathers the
// applies that the requests in flight have submitted (until every request in a
// solve has one pending, or a short window has passed), then launches them
// together on the batch's stream: the pair kernels of all on-the-fly problems
// as one grouped launch per kernel variant over the concatenated work lists
// (per problem the same work items, launch shape and partial sums as alone, so
// results do not depend on the mix), the gathers, reductions, projections,
// GEMVs and GEMMs of each problem back to back.  Events order the batch's
// stream after the request's input and the request's stream after the result.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "bem_internal.h"

namespace bem {
void apply_dense_multi_dispatch(bem_problem &p, const double2 *X, double2 *Y, int R, bool bf16);
}

struct bem_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    std::mutex mu;
    std::condition_variable cv;
    struct Job {
        bem_problem *p;
        int kind;
        const double2 *X;
        double2 *Y;
        int R;
        bool done = false;
        bem::Error err{BEM_OK, ""};
    };
    std::deque<Job *> pending;
    int in_solve = 0;          // attached problems inside a solve
    int attached = 0;
    bool stop = false;
    std::thread th;
    double window_s = 3e-4;    // longest wait for the other requests' applies
    // statistics: dispatches, jobs, grouped pair launches, of them with several
    // problems, largest group, pair work items launched grouped
    int64_t stats[6] = {0, 0, 0, 0, 0, 0};
};

namespace bem {

namespace {

void dispatch(bem_batch &b, std::vector<bem_batch::Job *> &jobs)
{
    hipStream_t s = b.stream;
    std::vector<hipStream_t> saved(jobs.size());
    for (size_t i = 0; i < jobs.size(); ++i) {
        bem_problem &p = *jobs[i]->p;
        BEM_HIP(hipStreamWaitEvent(s, p.batch_ready, 0));
        saved[i] = p.stream;
        p.stream = s;
    }
    struct Restore {
        std::vector<bem_batch::Job *> &j;
        std::vector<hipStream_t> &st;
        ~Restore()
        {
            for (size_t i = 0; i < j.size(); ++i) j[i]->p->stream = st[i];
        }
    } restore{jobs, saved};
    // on-the-fly applies: one round per right-hand side index, the pair kernels
    // of a round grouped by kernel variant
    int max_r = 0;
    for (auto *j : jobs)
        if (j->kind == BATCH_OTF) max_r = std::max(max_r, j->R);
    for (int r = 0; r < max_r; ++r) {
        std::vector<bem_batch::Job *> round;
        for (auto *j : jobs)
            if (j->kind == BATCH_OTF && j->R > r) round.push_back(j);
        for (auto *j : round) launch_gather(*j->p, j->X + int64_t(r) * j->p->N);
        std::vector<std::vector<bem_problem *>> groups(8);
        for (auto *j : round) groups[pair_variant(*j->p)].push_back(j->p);
        for (auto &g : groups)
            for (size_t k = 0; k < g.size(); k += PAIR_GROUP_MAX) {
                std::vector<bem_problem *> part(g.begin() + k, g.begin() + std::min(g.size(), k + PAIR_GROUP_MAX));
                launch_pairs_group(s, part);
                b.stats[2] += 1;
                if (part.size() > 1) b.stats[3] += 1;
                b.stats[4] = std::max<int64_t>(b.stats[4], int64_t(part.size()));
                for (auto *q : part) b.stats[5] += q->n_work;
            }
        for (auto *j : round) {
            launch_reduce(*j->p);
            launch_scatter(*j->p, j->X + int64_t(r) * j->p->N, j->Y + int64_t(r) * j->p->N, 3);
        }
    }
    for (auto *j : jobs) {
        bem_problem &p = *j->p;
        if (j->kind == BATCH_GEMV) {
            for (int r = 0; r < j->R; ++r) launch_gemv(p, j->X + int64_t(r) * p.N, j->Y + int64_t(r) * p.N);
        } else if (j->kind == BATCH_GEMM_BF16 || j->kind == BATCH_GEMM_F32) {
            apply_dense_multi_dispatch(p, j->X, j->Y, j->R, j->kind == BATCH_GEMM_BF16);
        } else if (j->kind == BATCH_HMATRIX) {
            hmatrix_apply(p, j->X, j->Y, j->R, false);
        }
        BEM_HIP(hipEventRecord(p.batch_done, s));
    }
}

void dispatcher(bem_batch *b)
{
    (void)hipSetDevice(b->device);
    AllocScope scope(b->stream);
    std::unique_lock<std::mutex> lk(b->mu);
    for (;;) {
        b->cv.wait(lk, [&] { return b->stop || !b->pending.empty(); });
        if (b->pending.empty()) break;   // stop requested and nothing left
        // wait for the other requests in a solve to submit, at most the window
        const auto deadline = std::chrono::steady_clock::now() + std::chrono::duration<double>(b->window_s);
        b->cv.wait_until(lk, deadline, [&] { return b->stop || int(b->pending.size()) >= b->in_solve; });
        std::vector<bem_batch::Job *> jobs(b->pending.begin(), b->pending.end());
        b->pending.clear();
        lk.unlock();
        Error err{BEM_OK, ""};
        try {
            dispatch(*b, jobs);
        } catch (const Error &e) {
            err = e;
        }
        lk.lock();
        b->stats[0] += 1;
        b->stats[1] += int64_t(jobs.size());
        for (auto *j : jobs) {
            j->err = err;
            j->done = true;
        }
        b->cv.notify_all();
    }
}

}  // namespace

void batch_apply(bem_problem &p, int kind, const double2 *X, double2 *Y, int R)
{
    bem_batch &b = *p.batch;
    BEM_HIP(hipEventRecord(p.batch_ready, p.stream));
    bem_batch::Job job{&p, kind, X, Y, R};
    {
        std::unique_lock<std::mutex> lk(b.mu);
        b.pending.push_back(&job);
        b.cv.notify_all();
        b.cv.wait(lk, [&] { return job.done; });
    }
    if (job.err.status != BEM_OK) throw job.err;
    BEM_HIP(hipStreamWaitEvent(p.stream, p.batch_done, 0));
}

void batch_detach(bem_problem &p)
{
    std::lock_guard<std::mutex> lk(p.batch->mu);
    p.batch->attached -= 1;
    p.batch = nullptr;
}

void batch_enter(bem_batch &b)
{
    std::lock_guard<std::mutex> lk(b.mu);
    b.in_solve += 1;
}

void batch_leave(bem_batch &b)
{
    std::lock_guard<std::mutex> lk(b.mu);
    b.in_solve -= 1;
    b.cv.notify_all();
}

}  // namespace bem

namespace {
thread_local std::string g_batch_error;
}

extern "C" {

bem_status bem_batch_create(int device, bem_batch **out)
{
    if (!out) return BEM_ERR_INVALID_ARG;
    *out = nullptr;
    auto *b = new bem_batch;
    b->device = device;
    try {
        BEM_HIP(hipSetDevice(device));
        BEM_HIP(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
    } catch (const bem::Error &e) {
        bem::set_error(e.msg);
        delete b;
        return e.status;
    }
    b->th = std::thread(bem::dispatcher, b);
    *out = b;
    return BEM_OK;
}

bem_status bem_batch_attach(bem_problem *p, bem_batch *b)
{
    if (!p) {
        bem::set_error("bem_batch_attach: NULL problem");
        return BEM_ERR_INVALID_ARG;
    }
    if (b && b->device != p->device) {
        bem::set_error("bem_batch_attach: the batch and the problem are on different devices");
        return BEM_ERR_INVALID_ARG;
    }
    try {
        BEM_HIP(hipSetDevice(p->device));
        if (p->batch) {
            std::lock_guard<std::mutex> lk(p->batch->mu);
            p->batch->attached -= 1;
        }
        p->batch = b;
        if (b) {
            if (!p->batch_ready) BEM_HIP(hipEventCreateWithFlags(&p->batch_ready, hipEventDisableTiming));
            if (!p->batch_done) BEM_HIP(hipEventCreateWithFlags(&p->batch_done, hipEventDisableTiming));
            std::lock_guard<std::mutex> lk(b->mu);
            b->attached += 1;
        }
    } catch (const bem::Error &e) {
        bem::set_error(e.msg);
        return e.status;
    }
    return BEM_OK;
}

bem_status bem_batch_set_window(bem_batch *b, double seconds)
{
    if (!b || !(seconds >= 0) || !(seconds <= 10)) {
        bem::set_error("bem_batch_set_window: need a batch and 0 <= seconds <= 10");
        return BEM_ERR_INVALID_ARG;
    }
    std::lock_guard<std::mutex> lk(b->mu);
    b->window_s = seconds;
    return BEM_OK;
}

bem_status bem_batch_stats(bem_batch *b, int64_t *out6)
{
    if (!b || !out6) {
        bem::set_error("bem_batch_stats: bad arguments");
        return BEM_ERR_INVALID_ARG;
    }
    std::lock_guard<std::mutex> lk(b->mu);
    for (int i = 0; i < 6; ++i) out6[i] = b->stats[i];
    return BEM_OK;
}

void bem_batch_destroy(bem_batch *b)
{
    if (!b) return;
    {
        std::lock_guard<std::mutex> lk(b->mu);
        b->stop = true;
        b->cv.notify_all();
    }
    if (b->th.joinable()) b->th.join();
    if (b->stream) {
        (void)hipSetDevice(b->device);
        (void)hipStreamSynchronize(b->stream);
        (void)hipStreamDestroy(b->stream);
    }
    delete b;
}

}  // extern "C"
