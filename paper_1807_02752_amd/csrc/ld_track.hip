// ld_track.hip -- lane tracking across frames: an alpha-beta filter on each lane's start
// column with greedy gated association (the reading taken for the tracker the paper names as
// future work in Sec. 4; the steps are listed at ld_track in ld.h).  One thread per frame,
// each folding its frame's lanes into its own stream's state in device memory; the work per
// frame is at most 16 x 16 distance tests per assignment round, so the launch is latency, not
// throughput, bound.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdint>

#include "ld.h"
#include "ld_internal.h"

namespace {

constexpr int kT = 64;
static_assert(sizeof(ld_track_state) == 464 && offsetof(ld_track_state, x) == 208, "ld_track_state layout");

template <typename Index>
__global__ __launch_bounds__(kT) void k_track(int nframes, const int32_t* nact, const ld_lanes* lanes,
                                              ld_track_state* states, const Index* state_index,
                                              ld_track_params P) {
    const int b = blockIdx.x * kT + threadIdx.x;
    const int nf = nact != nullptr ? min(*nact, nframes) : nframes;
    if (b >= nf) return;
    const int64_t si = state_index != nullptr ? (int64_t)state_index[b] : b;
    if (si < 0) return;
    ld_track_state* s = states + si;
    const ld_lanes& L = lanes[b];
    const bool valid = !(L.flags & (LD_FLAG_NOROAD | LD_FLAG_NOVP));
    const int nd = valid ? min(max(L.n, 0), LD_MAX_LANES) : 0;
    const int n = min(max(s->n, 0), LD_MAX_LANES);
    double xh[LD_MAX_LANES];
    int mt[LD_MAX_LANES], md[LD_MAX_LANES];
    for (int t = 0; t < LD_MAX_LANES; ++t) {
        xh[t] = t < n ? s->x[t] + s->dx[t] : 0.0;
        mt[t] = -1;
        md[t] = -1;
    }
    // greedy: the closest unassigned pair within the gate, ties to the lower slot, then lane
    for (;;) {
        int bt = -1, bd = -1;
        double best = 0.0;
        for (int t = 0; t < n; ++t) {
            if (mt[t] >= 0) continue;
            for (int d = 0; d < nd; ++d) {
                if (md[d] >= 0) continue;
                const double dist = fabs((double)L.u_start[d] - xh[t]);
                if (!(dist <= P.gate)) continue;
                if (bt < 0 || dist < best) { bt = t; bd = d; best = dist; }
            }
        }
        if (bt < 0) break;
        mt[bt] = bd;
        md[bd] = bt;
    }
    // filter, then drop the tracks past max_misses keeping the others' order
    int k = 0;
    for (int t = 0; t < n; ++t) {
        double x = xh[t], dx = s->dx[t];
        int hits = s->hits[t], misses = s->misses[t];
        if (mt[t] >= 0) {
            const double r = (double)L.u_start[mt[t]] - xh[t];
            x = xh[t] + P.alpha * r;
            dx = dx + P.beta * r;
            hits += 1;
            misses = 0;
        } else {
            misses += 1;
        }
        if (misses > P.max_misses) continue;
        s->id[k] = s->id[t];
        s->hits[k] = hits;
        s->misses[k] = misses;
        s->x[k] = x;
        s->dx[k] = dx;
        ++k;
    }
    // births from the unassigned detections, in lane order
    for (int d = 0; d < nd; ++d) {
        if (md[d] >= 0 || k >= LD_MAX_LANES) continue;
        s->id[k] = s->next_id++;
        s->hits[k] = 1;
        s->misses[k] = 0;
        s->x[k] = (double)L.u_start[d];
        s->dx[k] = 0.0;
        ++k;
    }
    s->n = k;
    s->frames += 1;
}

}  // namespace

extern "C" void ld_track_params_default(ld_track_params* tp) {
    if (!tp) return;
    tp->alpha = 0.5;
    tp->beta = 0.1;
    tp->gate = 24.0;
    tp->confirm = 3;
    tp->max_misses = 5;
}

extern "C" ld_status ld_track(ld_frame f, const ld_lanes* lanes, ld_track_state* states, const int32_t* state_index,
                              const ld_track_params* tp, void* hip_stream) {
    LdRange rr_("ld_track");
    ldi_frame_view V;
    if (!f || !lanes || !states || ldi_frame_get_view(f, &V) != LD_OK) return LD_E_INVAL;
    ld_track_params P;
    ld_track_params_default(&P);
    if (tp) P = *tp;
    if (!(P.alpha > 0.0 && P.alpha <= 1.0) || !(P.beta >= 0.0 && P.beta <= 1.0) || !(P.gate > 0.0) ||
        !std::isfinite(P.gate) || P.confirm < 1 || P.max_misses < 0)
        return LD_E_INVAL;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (V.active > 0)
        hipLaunchKernelGGL(k_track<int32_t>, dim3((V.active + kT - 1) / kT), dim3(kT), 0, st, V.active, V.nact, lanes,
                           states, state_index, P);
    if (hipGetLastError() != hipSuccess) return LD_E_HIP;
    return ldi_frame_set_last(f, hip_stream);
}

ld_status ldi_track_streams(ld_frame f, const ld_lanes* lanes, ld_track_state* states, const uint64_t* stream_ids,
                            hipStream_t st) {
    ldi_frame_view V;
    if (!f || !lanes || !states || !stream_ids || ldi_frame_get_view(f, &V) != LD_OK) return LD_E_INVAL;
    ld_track_params P;
    ld_track_params_default(&P);
    if (V.active > 0)
        hipLaunchKernelGGL(k_track<uint64_t>, dim3((V.active + kT - 1) / kT), dim3(kT), 0, st, V.active, V.nact, lanes,
                           states, stream_ids, P);
    return hipGetLastError() == hipSuccess ? LD_OK : LD_E_HIP;
}
