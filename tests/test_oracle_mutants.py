"""The oracle's pins catch planted mistakes.

Each mutant is the oracle built with one deliberately wrong expression (a
flipped sign, a dropped term, a transposed operand, a wrong threshold rule,
a wrong sort order, a wrong chain-rule factor; see the mutation hook in
oracle/tgo.cpp).  The fast pin tests run against each mutant in a child
process and must fail.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    1: "conic off-diagonal sign",
    2: "dilation dropped",
    3: "J W transposed",
    4: "quaternion rotation sign",
    5: "stop rule blends the stopping Gaussian",
    6: "backward drops the transmittance suffix term",
    7: "2-sigma instead of 3-sigma rectangle",
    8: "tile lists ignore depth order",
    9: "mean gradient uses W instead of W^T",
    10: "branch variants report T in the alpha column",
    11: "branch variants drop the T bg term",
    12: "lifting: depth from disparity without the focal length",
    13: "lifting: pixel corner instead of pixel centre",
    14: "lifting: camera rotation not transposed",
    15: "z-buffer: a point lands in the pixel whose centre is nearest",
    16: "z-buffer: the last point wins instead of the nearest",
    17: "normals: sign of one cross-product term",
    18: "normals: not turned toward the camera",
    19: "blending: bilinear taps around the pixel corner",
    20: "blending: cosine against the ray instead of the reversed ray",
    21: "blending: weight without the distance term",
}


@pytest.mark.slow
@pytest.mark.parametrize("plant", sorted(MUTANTS))
def test_pins_catch_planted_mistake(plant, tmp_path):
    sys.path.insert(0, ROOT)
    from oracle import build as obuild
    lib = obuild.build(out=str(tmp_path / f"libtgo_plant{plant}.so"), plant=plant)
    env = dict(os.environ, TGO_LIB_OVERRIDE=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_lift_pins.py"),
                        os.path.join(ROOT, "tests", "test_zsplat_pins.py"),
                        os.path.join(ROOT, "tests", "test_blend_pins.py"),
                        "-k", "not fd_cfg3_small"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {plant} ({MUTANTS[plant]}) survived the pins:\n{r.stdout[-2000:]}"
