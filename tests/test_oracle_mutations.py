"""The pins catch plausible mistakes: the oracle is rebuilt with one planted
mistake at a time (a slip in the reduced source, the scattering orientation,
the track weight, the attenuation, the estimator, the volumes, the
fission source, the azimuthal weights or the chain sweep) and the pin
suite must fail for every one of them."""
import os
import subprocess
import sys

import pytest

from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTATIONS = {
    1: "reduced source without 1/(4 pi)",
    2: "scattering matrix transposed",
    3: "track weight without sin(theta)",
    4: "linearised attenuation",
    5: "estimator without the 4 pi qhat term",
    6: "volumes from one sweep direction",
    7: "fission source without 1/k (eigenvalue mode)",
    8: "azimuthal weights from the desired angles",
    9: "chain sweep that drops the flux at reflective crossings",
}


@pytest.mark.parametrize("k", sorted(MUTATIONS))
def test_pins_fail_for_planted_mistake(k, tmp_path):
    lib = O.build(path=str(tmp_path / f"liboracle_m{k}.so"), mutation=k)
    env = dict(os.environ, MOC_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu", os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1, f"mutation {k} ({MUTATIONS[k]}) was not caught:\n{r.stdout[-2000:]}"
