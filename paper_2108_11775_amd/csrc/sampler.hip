// sampler.hip -- the PDMP producer/consumer (Sec. 3.3): a background diffeomorphic
// sampler keeps a bounded concurrent bucket S filled with morphed samples, and the
// planner's main thread draws from S without ever waiting -- when S is empty it
// draws from the prior instead, so a slow or failed GPU only reverts the planner to
// plain sampling.  Host code only (the GPU work goes through the morph entry points).
//
// Bucket: a single-producer single-consumer ring of `capacity` samples (a power of
// two) with acquire/release head and tail counters; the producer thread is the only
// writer, the consumer (the caller of pop) the only reader.
//
// Producer: one thread per sampler; batch b draws the Philox prior batch of stream
// (stream_id + b), morphs it on its own HIP stream (default priority), copies it to
// pinned host memory and pushes it, double-buffered so that the GPU works on batch
// b + 1 while batch b is pushed.  The pushed sample i of batch b carries the index
// b * batch + i.
//
// Prior fallback: the k-th fallback draw is sample k of the Philox prior of stream
// prior_stream_id (the same values pdmp_uniform_samples gives), so every draw is
// reproducible.
//
// RRT consumer: a plain RRT in the plane (Sec. 3.3's main thread in its simplest
// form): nearest node by linear scan, a fixed steering step, edges checked against
// discs in FP64, goal connection when the new node is within the goal tolerance.
#include "pdmp_common.h"

#include <atomic>
#include <chrono>
#include <cstring>
#include <thread>
#include <vector>

namespace pdmp {
namespace {

// ---------------------------------------------------------------- bucket ---

struct Bucket {
    int dim = 0;
    int64_t cap = 0, mask = 0;
    std::vector<float> data;  // [cap][dim]
    std::vector<int64_t> idx;
    alignas(64) std::atomic<int64_t> head{0};  // written by the producer
    alignas(64) std::atomic<int64_t> tail{0};  // written by the consumer

    void init(int d, int64_t capacity) {
        dim = d;
        cap = capacity;
        mask = capacity - 1;
        data.assign((size_t)cap * d, 0.0f);
        idx.assign((size_t)cap, 0);
    }
    int64_t size() const {
        return head.load(std::memory_order_acquire) - tail.load(std::memory_order_acquire);
    }
    // Push samples [start, n) of an SoA batch x [dim][ld] as far as space allows.
    int64_t push(const float *x, int64_t ld, int64_t start, int64_t n, int64_t base_index) {
        const int64_t h = head.load(std::memory_order_relaxed);
        const int64_t t = tail.load(std::memory_order_acquire);
        int64_t room = cap - (h - t);
        int64_t cnt = n - start < room ? n - start : room;
        for (int64_t j = 0; j < cnt; ++j) {
            const int64_t slot = (h + j) & mask;
            for (int k = 0; k < dim; ++k) data[(size_t)slot * dim + k] = x[(size_t)k * ld + start + j];
            idx[(size_t)slot] = base_index + start + j;
        }
        head.store(h + cnt, std::memory_order_release);
        return cnt;
    }
    bool pop(float *x, int64_t *index) {
        const int64_t t = tail.load(std::memory_order_relaxed);
        const int64_t h = head.load(std::memory_order_acquire);
        if (t == h) return false;
        const int64_t slot = t & mask;
        for (int k = 0; k < dim; ++k) x[k] = data[(size_t)slot * dim + k];
        if (index) *index = idx[(size_t)slot];
        tail.store(t + 1, std::memory_order_release);
        return true;
    }
};

// ------------------------------------------------------- host prior draw ---

void philox_host(uint32_t c[4], uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0], p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

// Sample i of the prior of (seed, stream) on the box, exactly as pdmp_uniform_samples.
void prior_draw(uint64_t seed, uint32_t sid, const float *lo, const float *hi, int dim, int64_t i,
                float *x) {
#pragma clang fp contract(off)
    for (int b = 0; b * 4 < dim; ++b) {
        uint32_t c[4] = {(uint32_t)i, (uint32_t)((uint64_t)i >> 32), (uint32_t)b, sid};
        philox_host(c, (uint32_t)seed, (uint32_t)(seed >> 32));
        for (int w = 0; w < 4 && b * 4 + w < dim; ++w) {
            const int k = b * 4 + w;
            const double u = (double)(c[w] >> 8) * (1.0 / 16777216.0);
            const double span = (double)hi[k] - (double)lo[k];
            x[k] = (float)((double)lo[k] + span * u);
        }
    }
}

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace
}  // namespace pdmp

using namespace pdmp;

struct pdmp_bucket {
    Bucket b;
};

struct pdmp_sampler {
    pdmp_occupancy occ;
    pdmp_sampler_opts o;
    Bucket bucket;
    int device = 0;
    std::thread th;
    std::atomic<bool> stop{false}, paused{false}, running{false};
    std::atomic<int32_t> status{PDMP_OK};
    char err[512] = "";  // producer's message, written before status is published
    std::atomic<int64_t> batches{0}, produced{0};
    std::atomic<double> busy_s{0.0};
    int64_t popped_bucket = 0, popped_prior = 0, prior_next = 0;  // consumer side
    double t_start = 0.0;
};

namespace {

void producer_main(pdmp_sampler *s) {
    const int dim = s->o.dim;
    const int64_t B = s->o.batch;
    hipStream_t st = nullptr;
    float *x0 = nullptr, *x1[2] = {nullptr, nullptr}, *h[2] = {nullptr, nullptr};
    hipEvent_t ev[2] = {nullptr, nullptr};
    auto fail = [&](hipError_t e, const char *what) {
        if (e != hipSuccess) {
            snprintf(s->err, sizeof(s->err), "sampler producer: %s: %s", what,
                     hipGetErrorString(e));
            s->status.store(PDMP_EDEVICE, std::memory_order_release);
            return true;
        }
        return false;
    };
    bool ok = !fail(hipSetDevice(s->device), "hipSetDevice") &&
              !fail(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "hipStreamCreate") &&
              !fail(hipMalloc(&x0, sizeof(float) * dim * B), "hipMalloc") &&
              !fail(hipMalloc(&x1[0], sizeof(float) * dim * B), "hipMalloc") &&
              !fail(hipMalloc(&x1[1], sizeof(float) * dim * B), "hipMalloc") &&
              !fail(hipHostMalloc(&h[0], sizeof(float) * dim * B, hipHostMallocDefault),
                    "hipHostMalloc") &&
              !fail(hipHostMalloc(&h[1], sizeof(float) * dim * B, hipHostMallocDefault),
                    "hipHostMalloc") &&
              !fail(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming), "hipEventCreate") &&
              !fail(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming), "hipEventCreate");
    // issue batch b into buffer b & 1
    auto issue = [&](int64_t b) -> bool {
        const int u = (int)(b & 1);
        int32_t r = pdmp_uniform_samples(s->o.seed, s->o.stream_id + (uint32_t)b, s->o.lo, s->o.hi,
                                         dim, B, x0, st);
        if (!r) r = pdmp_morph_samples(&s->occ, nullptr, x0, x1[u], B, s->o.T, s->o.eta, st);
        if (r) {
            // the message sits in this thread's error buffer: hand it to the consumer
            snprintf(s->err, sizeof(s->err), "sampler producer: %s", pdmp_last_error());
            s->status.store(r, std::memory_order_release);
            return false;
        }
        return !fail(hipMemcpyAsync(h[u], x1[u], sizeof(float) * dim * B, hipMemcpyDeviceToHost,
                                    st),
                     "hipMemcpyAsync") &&
               !fail(hipEventRecord(ev[u], st), "hipEventRecord");
    };
    int64_t b = 0;
    bool pending = false;
    while (ok && !s->stop.load(std::memory_order_acquire)) {
        if (s->paused.load(std::memory_order_acquire)) {
            std::this_thread::sleep_for(std::chrono::microseconds(200));
            continue;
        }
        const double t0 = now_s();
        if (!pending) {
            if (!(ok = issue(b))) break;
            pending = true;
        }
        if (!(ok = issue(b + 1))) break;  // the GPU works on the next batch meanwhile
        if (fail(hipEventSynchronize(ev[b & 1]), "hipEventSynchronize")) break;
        s->busy_s.store(s->busy_s.load() + (now_s() - t0));
        s->batches.fetch_add(1);
        const float *hb = h[b & 1];
        int64_t done = 0;
        while (done < B && !s->stop.load(std::memory_order_acquire)) {
            if (s->paused.load(std::memory_order_acquire)) {
                std::this_thread::sleep_for(std::chrono::microseconds(200));
                continue;
            }
            const int64_t k = s->bucket.push(hb, B, done, B, b * B);
            done += k;
            s->produced.fetch_add(k);
            if (k == 0) std::this_thread::sleep_for(std::chrono::microseconds(50));
        }
        ++b;  // batch b + 1 is in flight and becomes the next one to push
    }
    if (st) (void)hipStreamSynchronize(st);
    for (int u = 0; u < 2; ++u) {
        if (ev[u]) (void)hipEventDestroy(ev[u]);
        if (x1[u]) (void)hipFree(x1[u]);
        if (h[u]) (void)hipHostFree(h[u]);
    }
    if (x0) (void)hipFree(x0);
    if (st) (void)hipStreamDestroy(st);
    s->running.store(false);
}

bool pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

bool seg_hits_disc(double ax, double ay, double bx, double by, double cx, double cy, double r) {
#pragma clang fp contract(off)
    const double dx = bx - ax, dy = by - ay;
    const double len2 = dx * dx + dy * dy;
    double t = 0.0;
    if (len2 > 0.0) {
        t = ((cx - ax) * dx + (cy - ay) * dy) / len2;
        if (t < 0.0) t = 0.0;
        if (t > 1.0) t = 1.0;
    }
    const double px = ax + t * dx, py = ay + t * dy;
    const double ex = cx - px, ey = cy - py;
    return ex * ex + ey * ey <= r * r;
}

bool seg_free(const pdmp_rrt_opts *o, double ax, double ay, double bx, double by) {
    for (int k = 0; k < o->n_discs; ++k)
        if (seg_hits_disc(ax, ay, bx, by, o->disc_x[k], o->disc_y[k], o->disc_r[k])) return false;
    return true;
}

}  // namespace

extern "C" {

// ---- bucket (exposed for the concurrency tests) ----

int32_t pdmp_bucket_create(int32_t dim, int64_t capacity, pdmp_bucket **out) {
    PDMP_REQUIRE(out != nullptr, "out NULL");
    PDMP_REQUIRE(dim >= 1 && dim <= 16, "dim %d not in [1,16]", dim);
    PDMP_REQUIRE(pow2(capacity), "capacity must be a power of two");
    auto *b = new pdmp_bucket();
    b->b.init(dim, capacity);
    *out = b;
    return PDMP_OK;
}

int64_t pdmp_bucket_push(pdmp_bucket *b, const float *x, int64_t ld, int64_t start, int64_t n,
                         int64_t base_index) {
    if (!b || !x || start < 0 || n < start || ld < n) return -1;
    return b->b.push(x, ld, start, n, base_index);
}

int32_t pdmp_bucket_pop(pdmp_bucket *b, float *x, int64_t *index) {
    if (!b || !x) return -1;
    return b->b.pop(x, index) ? 1 : 0;
}

int64_t pdmp_bucket_size(const pdmp_bucket *b) { return b ? b->b.size() : -1; }

void pdmp_bucket_destroy(pdmp_bucket *b) { delete b; }

// ---- sampler ----

int32_t pdmp_sampler_create(const pdmp_occupancy *occ, const pdmp_sampler_opts *opts,
                            pdmp_sampler **out) {
    PDMP_REQUIRE(out != nullptr, "out NULL");
    PDMP_REQUIRE(opts != nullptr, "opts NULL");
    PDMP_REQUIRE(opts->dim == 2 || opts->dim == 3, "dim must be 2 or 3");
    PDMP_REQUIRE(opts->batch >= 1, "batch < 1");
    PDMP_REQUIRE(pow2(opts->capacity), "capacity must be a power of two");
    PDMP_REQUIRE(opts->T >= 0 && std::isfinite(opts->eta), "T/eta invalid");
    for (int k = 0; k < opts->dim; ++k)
        PDMP_REQUIRE(std::isfinite(opts->lo[k]) && std::isfinite(opts->hi[k]) &&
                         opts->lo[k] <= opts->hi[k],
                     "bad range on axis %d", k);
    PDMP_REQUIRE(occ == nullptr || occ->dim == opts->dim, "occupancy dim differs from opts dim");
    auto *s = new pdmp_sampler();
    if (occ) s->occ = *occ;
    else std::memset(&s->occ, 0, sizeof(s->occ));
    s->o = *opts;
    s->bucket.init(opts->dim, opts->capacity);
    *out = s;
    return PDMP_OK;
}

int32_t pdmp_sampler_start(pdmp_sampler *s) {
    PDMP_REQUIRE(s != nullptr, "sampler NULL");
    PDMP_REQUIRE(s->occ.hinges != nullptr, "the sampler has no occupancy (prior only)");
    PDMP_REQUIRE(!s->running.load(), "already running");
    if (s->th.joinable()) {
        // the producer ended on its own, which it does only on a failure: join it and
        // keep that failure visible instead of starting over
        s->th.join();
        const int32_t prev = s->status.load(std::memory_order_acquire);
        if (prev != PDMP_OK) {
            set_error("the producer stopped with an error, destroy the sampler (%s)", s->err);
            return PDMP_EINVAL;
        }
    }
    hipError_t e = hipGetDevice(&s->device);
    if (e != hipSuccess) {
        set_error("hipGetDevice: %s", hipGetErrorString(e));
        return PDMP_EDEVICE;
    }
    s->stop.store(false);
    s->running.store(true);
    s->t_start = now_s();
    s->th = std::thread(producer_main, s);
    return PDMP_OK;
}

int32_t pdmp_sampler_pause(pdmp_sampler *s, int32_t paused) {
    PDMP_REQUIRE(s != nullptr, "sampler NULL");
    s->paused.store(paused != 0, std::memory_order_release);
    return PDMP_OK;
}

int32_t pdmp_sampler_pop(pdmp_sampler *s, int64_t n, float *x, int64_t *index,
                         uint8_t *from_bucket) {
    PDMP_REQUIRE(s != nullptr, "sampler NULL");
    PDMP_REQUIRE(n >= 0 && (n == 0 || x), "x NULL");
    const int dim = s->o.dim;
    for (int64_t i = 0; i < n; ++i) {
        float *xi = x + (size_t)i * dim;
        int64_t id;
        if (s->bucket.pop(xi, &id)) {
            ++s->popped_bucket;
            if (from_bucket) from_bucket[i] = 1;
        } else {
            const int64_t k = s->prior_next++;
            prior_draw(s->o.seed, s->o.prior_stream_id, s->o.lo, s->o.hi, dim, k, xi);
            id = -1 - k;
            ++s->popped_prior;
            if (from_bucket) from_bucket[i] = 0;
        }
        if (index) index[i] = id;
    }
    return PDMP_OK;
}

int32_t pdmp_sampler_get_stats(const pdmp_sampler *s, pdmp_sampler_stats *st) {
    PDMP_REQUIRE(s && st, "NULL argument");
    st->batches = s->batches.load();
    st->produced = s->produced.load();
    st->popped_bucket = s->popped_bucket;
    st->popped_prior = s->popped_prior;
    st->bucket_size = s->bucket.size();
    st->status = s->status.load(std::memory_order_acquire);
    if (st->status != PDMP_OK) set_error("%s", s->err);
    st->running = s->running.load() ? 1 : 0;
    st->producer_busy_s = s->busy_s.load();
    st->elapsed_s = s->t_start > 0.0 ? now_s() - s->t_start : 0.0;
    return PDMP_OK;
}

int32_t pdmp_sampler_destroy(pdmp_sampler *s) {
    if (!s) return PDMP_OK;
    s->stop.store(true, std::memory_order_release);
    if (s->th.joinable()) s->th.join();
    const int32_t st = s->status.load(std::memory_order_acquire);
    if (st != PDMP_OK) set_error("%s", s->err);
    delete s;
    return st;
}

// ---- RRT consumer ----

int32_t pdmp_rrt_run(pdmp_sampler *s, const pdmp_rrt_opts *o, float *nodes, int32_t *parent,
                     float *samples, uint8_t *from_bucket, double *t_sample,
                     pdmp_rrt_result *res) {
#pragma clang fp contract(off)
    PDMP_REQUIRE(s != nullptr, "sampler NULL (use a sampler without occupancy for the prior)");
    PDMP_REQUIRE(o && nodes && parent && res, "NULL argument");
    PDMP_REQUIRE(s->o.dim == 2, "the RRT consumer is planar (dim 2)");
    PDMP_REQUIRE(o->max_iters >= 1 && o->step > 0.0f && std::isfinite(o->goal_tol),
                 "bad RRT options");
    PDMP_REQUIRE(o->n_discs == 0 || (o->disc_x && o->disc_y && o->disc_r), "disc arrays NULL");
    const double t0 = now_s();
    int32_t nn = 1;
    nodes[0] = o->start[0];
    nodes[1] = o->start[1];
    parent[0] = -1;
    std::memset(res, 0, sizeof(*res));
    int32_t it = 0;
    for (; it < o->max_iters; ++it) {
        if (o->time_budget_s > 0.0 && now_s() - t0 > o->time_budget_s) break;
        float q[2];
        int64_t id;
        uint8_t fb;
        pdmp_sampler_pop(s, 1, q, &id, &fb);
        if (samples) {
            samples[2 * it] = q[0];
            samples[2 * it + 1] = q[1];
        }
        if (from_bucket) from_bucket[it] = fb;
        if (t_sample) t_sample[it] = now_s() - t0;
        if (fb) ++res->from_bucket;
        else ++res->from_prior;
        // nearest node (squared distance in FP64; ties to the lowest index)
        int32_t best = 0;
        double bd = 0.0;
        for (int32_t j = 0; j < nn; ++j) {
            const double dx = (double)q[0] - (double)nodes[2 * j];
            const double dy = (double)q[1] - (double)nodes[2 * j + 1];
            const double d2 = dx * dx + dy * dy;
            if (j == 0 || d2 < bd) {
                bd = d2;
                best = j;
            }
        }
        const double px = nodes[2 * best], py = nodes[2 * best + 1];
        double nx = q[0], ny = q[1];
        const double dist = std::sqrt(bd);
        if (dist > (double)o->step) {
            nx = px + (double)o->step * (((double)q[0] - px) / dist);
            ny = py + (double)o->step * (((double)q[1] - py) / dist);
        }
        const float fx = (float)nx, fy = (float)ny;
        if (!seg_free(o, px, py, (double)fx, (double)fy)) continue;
        nodes[2 * nn] = fx;
        nodes[2 * nn + 1] = fy;
        parent[nn] = best;
        const int32_t added = nn++;
        const double gx = (double)o->goal[0] - (double)fx, gy = (double)o->goal[1] - (double)fy;
        if (o->goal_tol >= 0.0f &&
            gx * gx + gy * gy <= (double)o->goal_tol * (double)o->goal_tol &&
            seg_free(o, fx, fy, o->goal[0], o->goal[1])) {
            nodes[2 * nn] = o->goal[0];
            nodes[2 * nn + 1] = o->goal[1];
            parent[nn] = added;
            ++nn;
            res->solved = 1;
            ++it;
            break;
        }
    }
    res->iters = it;
    res->n_nodes = nn;
    res->elapsed_s = now_s() - t0;
    if (res->solved) {
        double len = 0.0;
        for (int32_t j = nn - 1; parent[j] >= 0; j = parent[j]) {
            const double dx = (double)nodes[2 * j] - (double)nodes[2 * parent[j]];
            const double dy = (double)nodes[2 * j + 1] - (double)nodes[2 * parent[j] + 1];
            len += std::sqrt(dx * dx + dy * dy);
        }
        res->path_len = len;
    }
    return PDMP_OK;
}

}  // extern "C"
