"""Projection quality (Supp. C) of the HIP path's UT: against Monte-Carlo
references of each particle's projected points, its median KL stays at the
sampling floor for pinhole, wide equidistant fisheye, distorted fisheye and
rolling-shutter cameras, and its per-particle KL equals the oracle UT's."""
import sys

import numpy as np
import pytest

import projection_quality as Q

pytestmark = pytest.mark.gpu


def test_gpu_ut_projection_quality_sweep():
    floor = Q.noise_floor_median()
    for name, sc, cam in Q.sweep():
        print(f"[projection quality] {name}", flush=True)
        vis_g, mg, cg = Q.ut_gpu(sc, cam)
        vis_o, mo, co = Q.ut_oracle(sc, cam)
        idx = np.nonzero(vis_g & vis_o)[0][:400]
        assert idx.size >= 300, name
        ok, mm, mc = Q.mc_reference(sc, idx, cam, seed=11)
        idx, mm, mc = idx[ok], mm[ok], mc[ok]
        kg = Q.kl_gauss2(mm, mc, mg[idx], cg[idx])
        ko = Q.kl_gauss2(mm, mc, mo[idx], co[idx])
        print(f"  n={idx.size} median KL gpu={np.median(kg):.3e} oracle={np.median(ko):.3e} "
              f"max |diff|={np.abs(kg - ko).max():.1e}", flush=True)
        sys.stdout.flush()
        assert 0.85 < np.median(kg) / floor < 1.2, name
        assert np.abs(kg - ko).max() < 1e-4, name
