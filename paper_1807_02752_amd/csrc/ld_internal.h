// ld_internal.h -- hooks between the frame objects (ld.hip) and the serving layer
// (ld_server.hip).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>
#include <stddef.h>
#include <stdint.h>

#include "ld.h"

// A roctx range named after an ABI call around its host part (argument checks and the
// enqueueing of its kernels; the kernels themselves run later on the caller's stream), so a
// marker trace (rocprofv3 --marker-trace) shows each call beside the kernels it launched.
struct LdRange {
    explicit LdRange(const char* name) noexcept { roctxRangePush(name); }
    ~LdRange() { roctxRangePop(); }
    LdRange(const LdRange&) = delete;
    LdRange& operator=(const LdRange&) = delete;
};

// Kernels of later launches on f skip the frames b >= *d_count (d_count: device int32,
// nullable to process every launched frame).  Lets one captured graph of a full batch serve
// partial batches.
ld_status ldi_frame_bind_count(ld_frame f, const int32_t* d_count);

// Device array of the fits of f: 2 per frame (road profile, then V_px).
const ld_fit* ldi_frame_fits(ld_frame f);

// Bytes of device scratch a frame object of this shape allocates.
size_t ldi_frame_bytes(int32_t width, int32_t height, int32_t batch, int32_t d_max);

// What the network kernels (ld_cnn.hip) need of a frame object.
#define LDI_MAX_BANDS 4
#define LDI_BAND_ROWS 16
typedef struct {
    int32_t W, H, fmt, d_max, batch, active, stage;
    double varpi;
    const double* tab;        /* batch x 6 x H: f, f', V_py, V_px, A_v, B_v */
    const int32_t* info;      /* batch x 8: flags, v_h, ... */
    uint8_t* lane_bits;       /* batch x LDI_MAX_BANDS x LDI_BAND_ROWS x W: network decisions */
    const int32_t* nact;      /* nullable active-frame count on the device */
    const ld_edge* edges;     /* batch x H x W: road edges of each row (after the edge kernel) */
    const int32_t* rowcnt;    /* batch x H: road edges per row */
} ldi_frame_view;

ld_status ldi_frame_get_view(ld_frame f, ldi_frame_view* v);

// Records `stream` as the one ld_sync of f waits for (work enqueued outside ld.hip).
ld_status ldi_frame_set_last(ld_frame f, void* stream);

// Marks that the band decisions of the frame were written on `stream` (after ld_vdisp).
ld_status ldi_frame_mark_bands(ld_frame f, int32_t n_bands, void* stream);

// First row of band k (0 = bottom) of a frame whose road starts at v_h, or -1 without bands.
__host__ __device__ inline int ldi_band_top(int v_h, int H, int n_bands, int k) {
    const int R = H - v_h;
    if (R < LDI_BAND_ROWS || n_bands < 1) return -1;
    return (H - LDI_BAND_ROWS) - ((R - LDI_BAND_ROWS) * k) / n_bands;
}

// Network decisions for the active frames of f into its band buffer (ld_cnn.hip).
// With sparse set (the edge kernel has run), only the column tiles whose band rows hold a
// voting road edge are evaluated; the others get zero decisions.
ld_status ldi_cnn_bits(ld_cnn n, ld_frame f, const uint8_t* grey, int64_t gp, const void* disp, int64_t dp,
                       float* prob_out, int sparse, hipStream_t st);
const ld_cnn_config* ldi_cnn_config(ld_cnn n);

// ld_track for the serving layer: frame b updates states[stream_ids[b]] with the default
// tracker parameters (stream ids < the state count, distinct within the launch).
ld_status ldi_track_streams(ld_frame f, const ld_lanes* lanes, ld_track_state* states, const uint64_t* stream_ids,
                            hipStream_t st);
