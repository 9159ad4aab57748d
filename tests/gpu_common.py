"""Helpers for the GPU parity tests (test infrastructure)."""
import math

import numpy as np

from paper_2004_13887_amd import inputs as I


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a - b))


def compare(tag, got, ref, keys=("p", "ur", "ut", "uf", "T"), base=None):
    """per-field relative L2 (and of the change from ``base`` if given)"""
    out = {}
    for k in keys:
        e = rel_l2(got[k], ref[k])
        line = f"{tag} {k}: relL2={e:.3e}"
        if base is not None:
            d = rel_l2(got[k] - base[k], ref[k] - base[k])
            line += f" (change relL2={d:.3e})"
            out[k + "_change"] = d
        print(line, flush=True)
        out[k] = e
    return out


# ragged small cases: a sector, a full sphere (poles + periodic phi), the
# workload used for parity and minimal sizes
def small_cases():
    return {
        "parity": I.WORKLOADS["parity"],
        "sector-ragged": I.Workload("sector-ragged", I.sector(13, 29, 37, math.radians(25) / 29,
                                                              math.radians(31) / 37),
                                    mach=1e-2, amplitude=0.5, steps=1, K=3, seed=77),
        "sphere-ragged": I.Workload("sphere-ragged", I.full_sphere(11, 22, 40), mach=1e-3,
                                    amplitude=0.5, steps=1, K=3, seed=78),
        "sector-min": I.Workload("sector-min", I.sector(3, 3, 3, 0.01, 0.01), mach=1e-2,
                                 amplitude=0.5, steps=1, K=2, seed=79),
        "sphere-min": I.Workload("sphere-min", I.full_sphere(3, 3, 3), mach=1e-2, amplitude=0.5,
                                 steps=1, K=2, seed=80),
        # phi lines split into a power-of-two number of 4-cell chunks (16, 2, 1)
        "sphere-chunks16": I.Workload("sphere-chunks16", I.full_sphere(9, 14, 64), mach=1e-3,
                                      amplitude=0.5, steps=1, K=3, seed=81),
        "sphere-chunks2": I.Workload("sphere-chunks2", I.full_sphere(4, 5, 8), mach=1e-2,
                                     amplitude=0.5, steps=1, K=2, seed=82),
        "sphere-chunks1": I.Workload("sphere-chunks1", I.full_sphere(3, 4, 4), mach=1e-2,
                                     amplitude=0.5, steps=1, K=2, seed=83),
    }
