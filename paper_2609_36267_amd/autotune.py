"""Autotuner for the schedule of the min-cost-flow passes.

Every increasing sequence of shortest-path windows yields the same exact
labels and the same optimal flow (Section II-C's bucket order only decides
which equal-cost optimum the paper's solver reaches first), and every stop
rule of a pass keeps successive shortest paths exact, so the schedule is a
pure speed knob. Its best value depends on the scene: broad zero-distance
plateaus favour few hop windows, long fault-crossing paths favour many, a
few passes that settle every deficit first pay off where most residues pair
up over short distances (the fault scene) but not where low-coherence
patches hold long paths, and searching from the demands once few units are
left avoids the plateaus that the earlier passes made tight around the
supplies. The tile shape (16, 32 or 64 columns of 1024 loops) changes how
far labels travel inside one visit, vertically or horizontally, and how many
tiles a frontier lists, never the labels. tune_schedule() times candidate schedules on sample jobs of a
workload through the C ABI and installs the fastest process-wide (ties keep
the earlier candidate, the default first).
"""
from __future__ import annotations

import time

from . import binding as ww

# (first_hop_window, first_distance_step[, full_passes, first_deficit_after
# [, reverse_below[, hop_growth[, tile_cols]]]]), missing fields 0
# (hop_growth 2, tile_cols 32);
# PAPER_SCHEDULE is the paper's pass schedule (Section II-C: eight full
# multi-source passes, then searches that stop at the first deficit)
PAPER_SCHEDULE = (64, 256, 8, 1)
CANDIDATES = [(64, 256), (16, 256), (512, 256), (64, 64), (16, 64), (512, 64), (64, 1024),
              (16, 1024), (512, 1024), (64, 256, 2, 0), (64, 256, 4, 0), PAPER_SCHEDULE,
              (64, 256, 0, 0, 1024), (64, 256, 2, 0, 1024), (64, 256, 4, 0, 1024),
              (64, 256, 8, 0, 1024), (512, 64, 0, 0, 1024),
              (64, 256, 0, 0, 1024, 8), (64, 256, 4, 0, 1024, 4), (64, 256, 4, 0, 1024, 6),
              (64, 256, 4, 0, 1024, 8), (64, 256, 4, 0, 1024, 16), (64, 256, 0, 0, 0, 8),
              (64, 1024, 4, 0, 1024, 8), (64, 1024, 0, 0, 1024, 8), (64, 256, 4, 0, 4096, 8),
              (64, 256, 4, 0, 1024, 8, 64), (64, 256, 4, 0, 1024, 8, 16),
              (64, 256, 0, 0, 1024, 8, 64), (64, 256, 0, 0, 1024, 8, 16),
              (64, 1024, 0, 0, 1024, 8, 64), (64, 1024, 0, 0, 1024, 8, 16)]

FIELDS = 7
# full_passes, first_deficit_after, reverse_below, hop_growth, tile_cols
DEFAULT_TAIL = (0, 0, 0, 2, 32)


def pad(c):
    """A candidate with its missing trailing fields set to their defaults
    (0, and 2 for hop_growth)."""
    c = tuple(c)
    return c + DEFAULT_TAIL[len(c) - 2:]


def tune_schedule(jobs, candidates=None, reps: int = 1, batch: bool = False):
    """jobs: list of (psi, coh, valid, looks) device tensors.  Times each
    candidate on all jobs (sequential plain calls, or one ww_unwrap_batch
    solve of all of them when batch is true), keeps the fastest, installs
    it process-wide and returns (best candidate, {candidate: seconds}).  A
    two-field candidate keeps the default stop rule.  Costs must agree
    across candidates (they are exact); a disagreement raises."""
    import torch
    cands = list(candidates or CANDIDATES)
    old = ww.get_mcf_params()
    timings, costs = {}, None
    try:
        for c in cands:
            ww.set_mcf_params(*pad(c))
            best = float("inf")
            for _ in range(max(1, reps)):
                torch.cuda.synchronize()
                t = time.perf_counter()
                if batch:
                    res, _ = ww.unwrap_batch(jobs, sched=pad(c))
                    got = [r[2] for r in res]
                else:
                    got = [ww.unwrap(*j[:3], j[3])[2] for j in jobs]
                torch.cuda.synchronize()
                best = min(best, time.perf_counter() - t)
            if costs is None:
                costs = got
            elif got != costs:
                raise RuntimeError(f"schedule {c} changed an optimal cost: {got} vs {costs}")
            timings[tuple(c)] = best
    except BaseException:
        ww.set_mcf_params(*old.as_tuple())
        raise
    choice = min(cands, key=lambda c: timings[tuple(c)])
    ww.set_mcf_params(*pad(choice))
    return choice, timings
