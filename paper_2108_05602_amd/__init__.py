"""MI355X (gfx950) single-pulse fringe search: HIP kernels behind a C ABI.

The compute path is libfringe.so (paper_2108_05602_amd/lib), built from
paper_2108_05602_amd/csrc by paper_2108_05602_amd.build; this package only
loads it (binding) and serves streamed chunks through it (serve).  There
is no CPU fallback: without the built library every entry point raises.
The library's host code turns candidate lists into single pulses and
positions (fringe_match, fringe_localize, fringe_delay_partials).
"""

from .binding import (CANDIDATE_DTYPE, PULSE_DTYPE, FRINGE_AUTOTUNE, FRINGE_DELAY_ONLY, FRINGE_DUMP_GRID, FRINGE_GRAPH, FRINGE_PLAIN, FRINGE_PROFILE, FRINGE_STREAMING, FringeError, Plan,
                      candidates_get, fringe_grid_get, fringe_last_error, fringe_plan,
                      fringe_plan_check, fringe_plan_destroy, fringe_plan_info, fringe_profile_get, fringe_search,
                      fringe_set_gains, fringe_set_shifts, fringe_dedisperse, fringe_match, fringe_localize,
                      fringe_delay_partials, fringe_autospectrum_gains, fringe_search_noalloc,
                      fringe_tune_load, fringe_tune_save, fringe_tune_clear, fringe_plan_tuning,
                      fringe_plan_set_chunk, fringe_plan_get_chunk,
                      fringe_strerror, fringe_window_id, fringe_windows_get, load)

__all__ = [
    "CANDIDATE_DTYPE", "PULSE_DTYPE", "FRINGE_AUTOTUNE", "FRINGE_DELAY_ONLY", "FRINGE_DUMP_GRID", "FRINGE_GRAPH", "FRINGE_PLAIN", "FRINGE_PROFILE", "FRINGE_STREAMING", "FringeError", "Plan",
    "candidates_get", "fringe_grid_get", "fringe_last_error", "fringe_plan",
    "fringe_plan_check", "fringe_plan_destroy", "fringe_plan_info", "fringe_profile_get", "fringe_search",
    "fringe_set_gains", "fringe_set_shifts", "fringe_dedisperse", "fringe_match", "fringe_localize",
    "fringe_delay_partials", "fringe_autospectrum_gains", "fringe_search_noalloc",
    "fringe_tune_load", "fringe_tune_save", "fringe_tune_clear", "fringe_plan_tuning",
    "fringe_plan_set_chunk", "fringe_plan_get_chunk",
    "fringe_strerror", "fringe_window_id", "fringe_windows_get", "load",
]
