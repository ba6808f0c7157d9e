// ld_internal.h -- hooks between the frame objects (ld.hip) and the serving layer
// (ld_server.hip).  Not part of the C ABI.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "ld.h"

// Kernels of later launches on f skip the frames b >= *d_count (d_count: device int32,
// nullable to process every launched frame).  Lets one captured graph of a full batch serve
// partial batches.
ld_status ldi_frame_bind_count(ld_frame f, const int32_t* d_count);

// Device array of the fits of f: 2 per frame (road profile, then V_px).
const ld_fit* ldi_frame_fits(ld_frame f);

// Bytes of device scratch a frame object of this shape allocates.
size_t ldi_frame_bytes(int32_t width, int32_t height, int32_t batch, int32_t d_max);
