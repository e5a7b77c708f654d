"""The batched cascade's URAD lane machine against the per-cell URAD
Newton, on the CPU: the device solver headers compiled for the host
(hipcc; no GPU needed) run both on every cascade cell of a seeded batch,
and the outputs must agree bit for bit.  The batch's explicit state comes
from the oracle's prim_to_cons."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_1312_6127_amd import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = shutil.which("hipcc")


@pytest.mark.skipif(HIPCC is None, reason="hipcc not found")
def test_urad_lane_machine_matches_per_cell_newton(orc, tmp_path):
    n = 6000
    pd, P, dt, ca, ce = I.implicit_batch(n, seed=9)
    g0 = orc.geom(pd, 0.0, 0.0)
    U = np.stack([orc.p2u(pd, g0, P[:, c]) for c in range(n)], axis=1)
    Ui = U.copy()
    Ui[8] *= 1.3
    Ui[1] -= 0.3 * U[8]
    fn = tmp_path / "batch.bin"
    with open(fn, "wb") as f:
        np.array([n], dtype=np.int64).tofile(f)
        np.array([pd["gam"], pd["arad"], pd["gamma_max"], pd["tol_pmhd"], pd["tol_urad"],
                  pd["tol_accept"], pd["tol_fail"], pd["max_iter"], pd["roundoff"], 0.0]).tofile(f)
        for a in (Ui, P, dt, ca, ce):
            np.ascontiguousarray(a, dtype=np.float64).tofile(f)
    exe = tmp_path / "urad_lane_check"
    subprocess.run([HIPCC, "-O2", "-std=c++17", "-x", "hip", "--offload-arch=gfx950",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-o", str(exe), os.path.join(HERE, "host", "urad_lane_check.cpp")],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe), str(fn)], check=True, capture_output=True, text=True).stdout
    vals = dict(zip(out.split()[0::2], map(int, out.split()[1::2])))
    assert vals["cascade"] > 1000 and vals["trips"] > 0
    assert vals["differing"] == 0, out
