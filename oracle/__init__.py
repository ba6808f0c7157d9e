"""CPU oracle of the lane-detection hot path -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this
package.  The GPU library never imports, links or calls it.
"""
from .ldref import (  # noqa: F401
    Params, band, band_top, bilateral, build, cand_mask, default_params, detect, detect_pruned, energy, fit, lib, m0m1, peaks,
    philox, ransac, TrackState, track_update,
    road_edges, road_tables, row_dp, sample, seed, sobel, stereo, stereo_stats, track_affine, vdisp_dp, vdisp_hist, votes, weights, window_dp,
)
