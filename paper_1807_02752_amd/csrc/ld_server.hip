// ld_server.hip -- continuous batching of lane-detection frames from many camera streams
// (see the serving section of ld.h).  Host-side scheduler plus two small device kernels that
// move per-stream state between the stream table and a batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <new>
#include <vector>

#include "ld.h"
#include "ld_internal.h"

namespace {

// Per-stream state kept in device memory between frames.
struct StreamState {
    double gamma_raw[5];   // last V_px fit, raw basis (NaN: none yet)
    int64_t frames;        // frames finished
};

// seed[i] = state[sid[i]].gamma_raw for the n active frames of a batch
__global__ void k_gather_seeds(const StreamState* st, const uint64_t* sid, const int32_t* nact, double* seed) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= *nact) return;
    const StreamState& s = st[sid[i]];
    for (int p = 0; p < 5; ++p) seed[5 * i + p] = s.gamma_raw[p];
}

// state[sid[i]] <- this batch's V_px fit (kept only when the fit succeeded)
__global__ void k_store_state(StreamState* st, const uint64_t* sid, const int32_t* nact, const ld_fit* fits) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= *nact) return;
    StreamState& s = st[sid[i]];
    const ld_fit& g = fits[2 * i + 1];
    if (g.ok)
        for (int p = 0; p < 5; ++p) s.gamma_raw[p] = g.raw[p];
    s.frames += 1;
}

__global__ void k_init_state(StreamState* st, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int p = 0; p < 5; ++p) st[i].gamma_raw[p] = __longlong_as_double(0x7ff8000000000000LL);
    st[i].frames = 0;
}

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int elem_size(int fmt) { return fmt == LD_DISP_U8 ? 1 : (fmt == LD_DISP_F32 ? 4 : 2); }

struct Request {
    int64_t id;
    int32_t stream;
    int32_t cls;
    const uint8_t* grey;
    int64_t gp;
    const void* disp;
    int64_t dp;
    int64_t frame_idx;
    double t_submit;
};

struct Engine {
    int cls = 0, B = 0, W = 0, H = 0, es = 1;
    ld_frame f = nullptr;
    hipStream_t st = nullptr;
    hipGraphExec_t exec = nullptr;
    bool busy = false;
    uint8_t* d_grey = nullptr;    // B x H x W staging
    uint8_t* d_disp = nullptr;    // B x H x W x es staging
    uint64_t* d_sid = nullptr;
    int64_t* d_fidx = nullptr;
    int32_t* d_nact = nullptr;
    double* d_seed = nullptr;
    ld_lanes* d_lanes = nullptr;
    uint64_t* h_sid = nullptr;    // pinned
    int64_t* h_fidx = nullptr;
    int32_t* h_nact = nullptr;
    ld_lanes* h_lanes = nullptr;
    hipEvent_t done = nullptr;
    std::vector<Request> reqs;
};

}  // namespace

struct ld_server_s {
    ld_server_config cfg;
    ld_params P;
    std::vector<Engine*> engines;
    std::deque<Request> queue[LD_MAX_CLASSES];
    std::deque<ld_server_result> finished;
    StreamState* d_state = nullptr;
    ld_track_state* d_tracks = nullptr;   // per stream, with config track
    std::vector<int64_t> next_frame;
    std::vector<int32_t> stream_cls;
    std::vector<uint8_t> in_flight;
    int64_t next_req = 0;
    int64_t bytes = 0;
    int32_t per_class[LD_MAX_CLASSES] = {0, 0, 0, 0};
    int64_t admitted = 0;    // engines created after ld_server_create
    int64_t evicted = 0;     // idle engines freed to admit another class
};

namespace {

size_t engine_bytes(const ld_server_config& c, int k) {
    const size_t B = (size_t)c.max_batch[k], H = (size_t)c.height[k], W = (size_t)c.width[k];
    const size_t staging = B * H * W * (1 + (size_t)elem_size(c.fmt[k]));
    const size_t small = B * (8 + 8 + 5 * 8 + sizeof(ld_lanes)) + 64;
    return ldi_frame_bytes(c.width[k], c.height[k], c.max_batch[k], c.d_max[k]) + staging + small + 4096;
}

// Device memory kept free beyond an engine's own bytes when an engine is admitted.
constexpr int64_t kReserveBytes = (int64_t)512 << 20;

// An engine of class k fits the caller's budget and the device's free memory now.
bool can_admit(ld_server s, int k) {
    const int64_t need = (int64_t)engine_bytes(s->cfg, k);
    if (s->bytes + need > s->cfg.hbm_budget) return false;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return (int64_t)free_b >= need + kReserveBytes;
}

void free_engine(Engine* e) {
    if (!e) return;
    if (e->st) (void)hipStreamSynchronize(e->st);
    if (e->exec) (void)hipGraphExecDestroy(e->exec);
    if (e->f) (void)ld_frame_destroy(e->f);
    (void)hipFree(e->d_grey);
    (void)hipFree(e->d_disp);
    (void)hipFree(e->d_sid);
    (void)hipFree(e->d_fidx);
    (void)hipFree(e->d_nact);
    (void)hipFree(e->d_seed);
    (void)hipFree(e->d_lanes);
    (void)hipHostFree(e->h_sid);
    (void)hipHostFree(e->h_fidx);
    (void)hipHostFree(e->h_nact);
    (void)hipHostFree(e->h_lanes);
    if (e->done) (void)hipEventDestroy(e->done);
    if (e->st) (void)hipStreamDestroy(e->st);
    delete e;
}

// The device part of one batch, enqueued on the engine's stream: seeds from the stream
// table, the four steps (or the pruned path with the server's network), the state update and
// the copy of the lanes to pinned memory.
ld_status enqueue_batch_body(ld_server s, Engine* e) {
    const int B = e->B;
    const int64_t gp = e->W, dpt = (int64_t)e->W * e->es;
    ld_status r = LD_OK;
    const bool seed = s->cfg.seed_from_state != 0;
    if (seed)
        hipLaunchKernelGGL(k_gather_seeds, dim3((B + 63) / 64), dim3(64), 0, e->st, s->d_state, e->d_sid, e->d_nact,
                           e->d_seed);
    if (s->cfg.cnn) {
        r = ld_detect_pruned(e->f, s->cfg.cnn, e->d_grey, gp, e->d_disp, dpt, e->d_sid, e->d_fidx,
                             seed ? e->d_seed : nullptr, e->d_lanes, nullptr, e->st);
    } else {
        r = ld_vdisp(e->f, e->d_disp, dpt, e->d_sid, e->d_fidx, nullptr, nullptr, e->st);
        if (r == LD_OK)
            r = ld_vp_ransac(e->f, e->d_grey, gp, e->d_disp, dpt, e->d_sid, e->d_fidx, seed ? e->d_seed : nullptr, nullptr,
                             e->st);
        if (r == LD_OK) r = ld_lane_energy(e->f, nullptr, nullptr, e->st);
        if (r == LD_OK) r = ld_peaks(e->f, e->d_lanes, nullptr, e->st);
    }
    if (r != LD_OK) return r;
    hipLaunchKernelGGL(k_store_state, dim3((B + 63) / 64), dim3(64), 0, e->st, s->d_state, e->d_sid, e->d_nact, ldi_frame_fits(e->f));
    if (hipGetLastError() != hipSuccess) return LD_E_HIP;
    if (s->d_tracks) return ldi_track_streams(e->f, e->d_lanes, s->d_tracks, e->d_sid, e->st);
    return LD_OK;
}

ld_status make_engine(ld_server s, int k, Engine** out) {
    const ld_server_config& c = s->cfg;
    Engine* e = new (std::nothrow) Engine();
    if (!e) return LD_E_NOMEM;
    e->cls = k; e->B = c.max_batch[k]; e->W = c.width[k]; e->H = c.height[k]; e->es = elem_size(c.fmt[k]);
    const size_t B = e->B, H = e->H, W = e->W;
    ld_status st = ld_frame_create(e->W, e->H, e->B, c.fmt[k], c.d_max[k], &s->P, &e->f);
    if (st != LD_OK) { free_engine(e); return st; }
    bool ok = hipStreamCreateWithFlags(&e->st, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&e->done, hipEventDisableTiming) == hipSuccess &&
              hipMalloc(&e->d_grey, B * H * W) == hipSuccess && hipMalloc(&e->d_disp, B * H * W * e->es) == hipSuccess &&
              hipMalloc(&e->d_sid, B * 8) == hipSuccess && hipMalloc(&e->d_fidx, B * 8) == hipSuccess &&
              hipMalloc(&e->d_nact, 64) == hipSuccess && hipMalloc(&e->d_seed, B * 5 * 8) == hipSuccess &&
              hipMalloc(&e->d_lanes, B * sizeof(ld_lanes)) == hipSuccess &&
              hipHostMalloc(&e->h_sid, B * 8) == hipSuccess && hipHostMalloc(&e->h_fidx, B * 8) == hipSuccess &&
              hipHostMalloc(&e->h_nact, 64) == hipSuccess && hipHostMalloc(&e->h_lanes, B * sizeof(ld_lanes)) == hipSuccess;
    if (!ok) { (void)hipGetLastError(); free_engine(e); return LD_E_NOMEM; }
    // inputs of an empty engine are defined: zero frames, stream 0, count 0
    ok = hipMemsetAsync(e->d_grey, 0, B * H * W, e->st) == hipSuccess &&
         hipMemsetAsync(e->d_disp, 0, B * H * W * e->es, e->st) == hipSuccess &&
         hipMemsetAsync(e->d_sid, 0, B * 8, e->st) == hipSuccess && hipMemsetAsync(e->d_fidx, 0, B * 8, e->st) == hipSuccess &&
         hipMemsetAsync(e->d_nact, 0, 64, e->st) == hipSuccess && hipStreamSynchronize(e->st) == hipSuccess;
    if (!ok || ldi_frame_bind_count(e->f, e->d_nact) != LD_OK) { free_engine(e); return LD_E_HIP; }
    if (c.use_graphs) {
        // warm the kernels once eagerly (sets launch attributes), then capture the body
        if (enqueue_batch_body(s, e) != LD_OK || hipStreamSynchronize(e->st) != hipSuccess) { free_engine(e); return LD_E_HIP; }
        hipGraph_t g = nullptr;
        if (hipStreamBeginCapture(e->st, hipStreamCaptureModeThreadLocal) != hipSuccess) { free_engine(e); return LD_E_HIP; }
        const ld_status body = enqueue_batch_body(s, e);
        const hipError_t endc = hipStreamEndCapture(e->st, &g);
        if (body != LD_OK || endc != hipSuccess || hipGraphInstantiate(&e->exec, g, nullptr, nullptr, 0) != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            (void)hipGetLastError();
            free_engine(e);
            return LD_E_HIP;
        }
        (void)hipGraphDestroy(g);
    }
    *out = e;
    return LD_OK;
}

// Start one batch on an idle engine of class k from the queue (FIFO, one frame per stream).
bool start_batch(ld_server s, Engine* e) {
    std::deque<Request>& q = s->queue[e->cls];
    e->reqs.clear();
    for (auto it = q.begin(); it != q.end() && (int)e->reqs.size() < e->B;) {
        bool taken = s->in_flight[it->stream] != 0;
        for (const Request& r : e->reqs) taken = taken || r.stream == it->stream;
        if (!taken) {
            e->reqs.push_back(*it);
            it = q.erase(it);
        } else {
            ++it;
        }
    }
    if (e->reqs.empty()) return false;
    const int n = (int)e->reqs.size();
    const size_t H = e->H, W = e->W;
    for (int i = 0; i < n; ++i) {
        const Request& r = e->reqs[i];
        (void)hipMemcpy2DAsync(e->d_grey + (size_t)i * H * W, W, r.grey, r.gp, W, H, hipMemcpyDeviceToDevice, e->st);
        (void)hipMemcpy2DAsync(e->d_disp + (size_t)i * H * W * e->es, W * e->es, r.disp, r.dp, W * e->es, H,
                               hipMemcpyDeviceToDevice, e->st);
        e->h_sid[i] = (uint64_t)r.stream;
        e->h_fidx[i] = r.frame_idx;
        s->in_flight[r.stream] = 1;
    }
    *e->h_nact = n;
    (void)hipMemcpyAsync(e->d_sid, e->h_sid, (size_t)n * 8, hipMemcpyHostToDevice, e->st);
    (void)hipMemcpyAsync(e->d_fidx, e->h_fidx, (size_t)n * 8, hipMemcpyHostToDevice, e->st);
    (void)hipMemcpyAsync(e->d_nact, e->h_nact, 4, hipMemcpyHostToDevice, e->st);
    if (e->exec) {
        (void)hipGraphLaunch(e->exec, e->st);
    } else {
        (void)enqueue_batch_body(s, e);
    }
    (void)hipMemcpyAsync(e->h_lanes, e->d_lanes, (size_t)n * sizeof(ld_lanes), hipMemcpyDeviceToHost, e->st);
    (void)hipEventRecord(e->done, e->st);
    e->busy = true;
    return true;
}

}  // namespace

extern "C" {

ld_status ld_server_create(const ld_server_config* cfg, const ld_params* p, ld_server* out) {
    if (!cfg || !out) return LD_E_INVAL;
    *out = nullptr;
    const ld_server_config& c = *cfg;
    if (c.n_classes < 1 || c.n_classes > LD_MAX_CLASSES || c.n_streams < 1 || c.n_streams > (1 << 20) ||
        c.inflight < 1 || c.inflight > 8 || c.max_queue < 1 || c.hbm_budget < 0 || (c.track != 0 && c.track != 1))
        return LD_E_INVAL;
    for (int k = 0; k < c.n_classes; ++k) {
        if (c.width[k] < 8 || c.width[k] > 4096 || c.height[k] < 8 || c.height[k] > 4096 || c.fmt[k] < 0 ||
            c.fmt[k] > 2 || c.d_max[k] < 1 || c.d_max[k] > 1023 || c.max_batch[k] < 1 || c.max_batch[k] > 4096)
            return LD_E_INVAL;
    }
    ld_server s = new (std::nothrow) ld_server_s();
    if (!s) return LD_E_NOMEM;
    s->cfg = c;
    ld_params_default(&s->P);
    if (p) s->P = *p;
    s->next_frame.assign(c.n_streams, 0);
    s->stream_cls.assign(c.n_streams, -1);
    s->in_flight.assign(c.n_streams, 0);
    if (hipMalloc(&s->d_state, sizeof(StreamState) * (size_t)c.n_streams) != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        return LD_E_NOMEM;
    }
    hipLaunchKernelGGL(k_init_state, dim3((c.n_streams + 255) / 256), dim3(256), 0, nullptr, s->d_state, c.n_streams);
    if (c.track) {
        const size_t tb = sizeof(ld_track_state) * (size_t)c.n_streams;
        if (hipMalloc(&s->d_tracks, tb) != hipSuccess || hipMemset(s->d_tracks, 0, tb) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipFree(s->d_tracks);
            (void)hipFree(s->d_state);
            delete s;
            return LD_E_NOMEM;
        }
    }
    if (hipDeviceSynchronize() != hipSuccess) {
        (void)hipFree(s->d_tracks);
        (void)hipFree(s->d_state);
        delete s;
        return LD_E_HIP;
    }
    // engines: round-robin over the classes while the budget allows
    bool grew = true;
    for (int round = 0; round < c.inflight && grew; ++round) {
        grew = false;
        for (int k = 0; k < c.n_classes; ++k) {
            const int64_t need = (int64_t)engine_bytes(c, k);
            if (!can_admit(s, k)) continue;
            Engine* e = nullptr;
            const ld_status st = make_engine(s, k, &e);
            if (st == LD_E_NOMEM) continue;
            if (st != LD_OK) { ld_server_destroy(s); return st; }
            s->engines.push_back(e);
            s->bytes += need;
            s->per_class[k] += 1;
            grew = true;
        }
    }
    *out = s;
    return LD_OK;
}

ld_status ld_server_destroy(ld_server s) {
    if (!s) return LD_OK;
    for (Engine* e : s->engines) free_engine(e);
    (void)hipFree(s->d_state);
    (void)hipFree(s->d_tracks);
    delete s;
    return LD_OK;
}

ld_status ld_server_submit(ld_server s, int32_t stream_id, int32_t cls, const uint8_t* grey, int64_t grey_pitch,
                           const void* disp, int64_t disp_pitch, int64_t* req_out) {
    LdRange rr_("ld_server_submit");
    if (!s || !grey || !disp || cls < 0 || cls >= s->cfg.n_classes || stream_id < 0 || stream_id >= s->cfg.n_streams)
        return LD_E_INVAL;
    const int W = s->cfg.width[cls], es = elem_size(s->cfg.fmt[cls]);
    if (grey_pitch < W || disp_pitch < (int64_t)W * es) return LD_E_INVAL;
    if (s->stream_cls[stream_id] >= 0 && s->stream_cls[stream_id] != cls) return LD_E_INVAL;   // a stream keeps its size
    if ((int64_t)engine_bytes(s->cfg, cls) > s->cfg.hbm_budget) return LD_E_NOMEM;          // never admissible
    if ((int)s->queue[cls].size() >= s->cfg.max_queue) return LD_E_BUSY;
    s->stream_cls[stream_id] = cls;
    Request r;
    r.id = s->next_req++;
    r.stream = stream_id;
    r.cls = cls;
    r.grey = grey;
    r.gp = grey_pitch;
    r.disp = disp;
    r.dp = disp_pitch;
    r.frame_idx = s->next_frame[stream_id]++;
    r.t_submit = now_s();
    s->queue[cls].push_back(r);
    if (req_out) *req_out = r.id;
    return LD_OK;
}

ld_status ld_server_poll(ld_server s, ld_server_result* results, int32_t max_results, int32_t* n_out) {
    LdRange rr_("ld_server_poll");
    if (!s || (max_results > 0 && !results) || !n_out) return LD_E_INVAL;
    ld_status status = LD_OK;
    // 1. retire finished batches
    for (Engine* e : s->engines) {
        if (!e->busy) continue;
        const hipError_t q = hipEventQuery(e->done);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) status = LD_E_HIP;
        const double t = now_s();
        for (size_t i = 0; i < e->reqs.size(); ++i) {
            const Request& r = e->reqs[i];
            ld_server_result res;
            res.request = r.id;
            res.stream_id = r.stream;
            res.cls = r.cls;
            res.frame_idx = r.frame_idx;
            res.t_submit = r.t_submit;
            res.t_done = t;
            res.lanes = e->h_lanes[i];
            s->finished.push_back(res);
            s->in_flight[r.stream] = 0;
        }
        e->reqs.clear();
        e->busy = false;
    }
    // 2. start batches on idle engines
    for (Engine* e : s->engines)
        if (!e->busy && !s->queue[e->cls].empty()) start_batch(s, e);
    // 3. admission: a class with waiting requests and no idle engine gets a new engine when its
    // bytes fit the budget and the free device memory; a class with no engine at all may take the
    // place of idle engines of classes that have nothing queued
    for (int k = 0; k < s->cfg.n_classes; ++k) {
        if (s->queue[k].empty()) continue;
        bool idle = false;
        for (Engine* e : s->engines) idle = idle || (e->cls == k && !e->busy);
        if (idle || s->per_class[k] >= s->cfg.inflight) continue;
        if (s->per_class[k] == 0) {
            for (size_t i = 0; i < s->engines.size() && !can_admit(s, k);) {
                Engine* e = s->engines[i];
                if (!e->busy && e->cls != k && s->queue[e->cls].empty()) {
                    s->bytes -= (int64_t)engine_bytes(s->cfg, e->cls);
                    s->per_class[e->cls] -= 1;
                    free_engine(e);
                    s->engines.erase(s->engines.begin() + (ptrdiff_t)i);
                    s->evicted += 1;
                } else {
                    ++i;
                }
            }
        }
        if (!can_admit(s, k)) continue;
        Engine* e = nullptr;
        const ld_status st = make_engine(s, k, &e);
        if (st == LD_E_NOMEM) continue;
        if (st != LD_OK) { status = st; continue; }
        s->engines.push_back(e);
        s->bytes += (int64_t)engine_bytes(s->cfg, k);
        s->per_class[k] += 1;
        s->admitted += 1;
        start_batch(s, e);
    }
    if (hipGetLastError() != hipSuccess) status = LD_E_HIP;
    // 4. hand out results
    int n = 0;
    while (n < max_results && !s->finished.empty()) {
        results[n++] = s->finished.front();
        s->finished.pop_front();
    }
    *n_out = n;
    return status;
}

ld_status ld_server_pending(ld_server s, int32_t* queued, int32_t* inflight) {
    if (!s) return LD_E_INVAL;
    int q = 0, f = 0;
    for (int k = 0; k < s->cfg.n_classes; ++k) q += (int)s->queue[k].size();
    for (Engine* e : s->engines) f += (int)e->reqs.size();
    f += (int)s->finished.size();
    if (queued) *queued = q;
    if (inflight) *inflight = f;
    return LD_OK;
}

ld_status ld_server_tracks(ld_server s, int32_t stream_id, ld_track_state* out) {
    if (!s || !out || stream_id < 0 || stream_id >= s->cfg.n_streams) return LD_E_INVAL;
    if (!s->d_tracks) return LD_E_STATE;
    // the engines' streams are non-blocking: wait for the batches in flight first
    for (Engine* e : s->engines)
        if (hipStreamSynchronize(e->st) != hipSuccess) return LD_E_HIP;
    return hipMemcpy(out, s->d_tracks + stream_id, sizeof(ld_track_state), hipMemcpyDeviceToHost) == hipSuccess
               ? LD_OK : LD_E_HIP;
}

ld_status ld_server_engines(ld_server s, int32_t* per_class, int64_t* bytes) {
    if (!s) return LD_E_INVAL;
    if (per_class)
        for (int k = 0; k < LD_MAX_CLASSES; ++k) per_class[k] = s->per_class[k];
    if (bytes) *bytes = s->bytes;
    return LD_OK;
}

}  // extern "C"
