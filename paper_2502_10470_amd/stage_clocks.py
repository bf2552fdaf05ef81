"""Cycles per stage of the generation kernels, from a diagnostic build.

    python -m paper_2502_10470_amd.stage_clocks build       # libmetade_stage.so
    python -m paper_2502_10470_amd.stage_clocks c3 c4 c4bf16
    python -m paper_2502_10470_amd.stage_clocks --all-waves c3     # every wave

The diagnostic build compiles the library with -DMDE_STAGE_CLOCKS: every wave
of a generation kernel reads clock64 after each barrier and adds the cycles
since the previous read to a per-(block, wave, stage) total, written to a
device array at the end of the launch (ordinary builds contain none of it).
Every wave, producers included, also reads it just before each barrier: the
cycles from the previous barrier to that point are the wave's own work in
the stage, the rest of the stage its wait for the others.
The runs: the D = 20 executor launch of full MetaDE (64 runs, the first
evolver generation's theta from the library's own evolver, 1000 generations,
tuned part count) and the D = 100 launch (128 runs x N = 256, 500
generations) in the plain and the bf16 precision.  Printed: the launch time
and, per listed wave, the mean over the runs of the cycles per generation in
each stage.
"""
from __future__ import annotations

import ctypes
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
STAGE_LIB = os.path.join(HERE, "libmetade_stage.so")
SB, SW, SN = 256, 16, 16   # blocks, waves per block and stage slots recorded (device.h)

LANE_STAGES = ["commit+draws", "ranking", "trials", "fitness",
               "work:commit", "work:ranking", "work:trials", "work:fitness"]
MFMA_STAGES = ["commit+draws", "ranking", "top-p", "trials", "rotation", "screen",
               "candidates", "re-evaluation", "work:commit", "work:ranking", "work:top-p",
               "work:trials", "work:rotation", "work:screen", "work:candidates",
               "work:re-evaluation"]


def build() -> str:
    from paper_2502_10470_amd.build import build as _build
    return _build(verbose=True, defines=("MDE_STAGE_CLOCKS",), tag="stage")


def _clocks(L, which: int) -> np.ndarray:
    a = np.zeros(SB * SW * SN, np.uint64)
    if L.metade_debug_stage_clocks(which, a.ctypes.data, a.nbytes) != 0:
        raise RuntimeError("metade_debug_stage_clocks failed")
    return a.reshape(SB, SW, SN).astype(np.float64)


def _report(L, name, which, n_blocks, G, waves, labels):
    n_int = sum(not x.startswith("work:") for x in labels)   # barrier-to-barrier stages
    c = _clocks(L, which)[:n_blocks] / G
    print(f"== {name}: cycles per generation, mean over {n_blocks} runs; "
          f"total per wave {c[:, waves[0], :n_int].sum(axis=1).mean():.0f}")
    for w in waves:
        row = c[:, w, :].mean(axis=0)
        print(f"  wave {w:2d}: " + "  ".join(f"{labels[k]} {row[k]:.0f}"
                                             for k in range(len(labels))))


def main(names, all_waves: bool = False) -> None:
    if not os.path.exists(STAGE_LIB):
        raise SystemExit(f"{STAGE_LIB} is missing: run `python -m {__package__}.stage_clocks build`")
    sys.path.insert(0, ROOT)
    from paper_2502_10470_amd import metade as M
    M.LIB_PATH = STAGE_LIB
    import torch
    import workloads as W
    from paper_2502_10470_amd import Batch

    L = M.lib()
    L.metade_debug_stage_clocks.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t]
    table = os.path.join(HERE, "tuning_gfx950.txt")
    for name in names:
        if name == "c3":
            wl = W.workload_c3()
            b = Batch(wl)
            b.outer_reset()
            b.outer_step(1, 1)
            b.set_theta(b.get_outer()[2].copy())
            b.reset()
            b.autotune(wl.G, table)
            G, which, waves, labels = wl.G, 0, [0, 4, 8, 12], LANE_STAGES
        elif name in ("c4", "c4bf16"):
            wl = W.workload_c4()
            b = Batch(wl, precision=M.BF16_REFINE if name == "c4bf16" else M.FP32)
            b.autotune(wl.G, table)
            G, which, waves, labels = wl.G, 1, [0, 7, 8, 11], MFMA_STAGES
        else:
            raise SystemExit(f"unknown workload {name!r} (c3, c4, c4bf16)")
        b.reset()
        b.kernel_timing(True)
        b.inner_step(G)
        ms, _ = b.kernel_time()
        b.kernel_timing(False)
        torch.cuda.synchronize()
        print(f"{name}: launch {ms:.2f} ms for {G} generations", flush=True)
        if all_waves:
            waves = list(range(SW))
        _report(L, name, which, wl.n_runs, G, waves, labels)
        sys.stdout.flush()
        b.close()


if __name__ == "__main__":
    args = sys.argv[1:]
    all_waves = "--all-waves" in args
    args = [a for a in args if a != "--all-waves"] or ["c3", "c4", "c4bf16"]
    if args == ["build"]:
        print(build())
    else:
        main(args, all_waves)
