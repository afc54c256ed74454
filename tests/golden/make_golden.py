"""Write the oracle regression fixtures in this folder (run from the repository root:
python tests/golden/make_golden.py). Every value comes from the oracle alone, on seeded inputs
from fv_inputs; the fixtures guard the oracle against unnoticed changes of its arithmetic (a
deliberate change regenerates them, in a commit naming the passage or reading behind it). They
are not pins: the pins are the tests of the oracle against exact solutions and invariants."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import fv_inputs as fi  # noqa: E402
import oracle as O  # noqa: E402


def cases():
    """(name, description, values) for each fixture case; values a flat float64 array."""
    out = []
    p = O.Problem(dim=1, n=(64,), eq="euler", flux="rusanov", integrator="forward_euler",
                  bc=("transmissive",))
    U, *_ = O.evolve(p, fi.sod_state(64), 0.1, 0.45)
    out.append(("sod_rusanov_first_order_64", "Sod, 64 cells, Rusanov, first order, forward Euler, CFL 0.45, t = 0.1", U))
    c, phi = fi.kh_coefficients(1912, [0])
    p = O.Problem(dim=2, n=(16, 16), eq="euler", flux="hllc", recon="weno3", integrator="ssprk3")
    U, *_ = O.evolve(p, fi.kh2d_state(16, c, phi), 10.0, 0.4, max_steps=5)
    out.append(("kh_weno3_hllc_ssprk3_16", "Kelvin-Helmholtz 16x16 (seed 1912, sample 0), WENO3 + HLLC + SSP-RK3, 5 steps, CFL 0.4", U))
    p = O.Problem(dim=1, n=(32,), eq="euler", flux="godunov", recon="muscl_minmod",
                  integrator="ssprk2", bc=("transmissive",))
    U, *_ = O.evolve(p, fi.sod_state(32), 0.1, 0.45)
    out.append(("sod_godunov_muscl_32", "Sod, 32 cells, Godunov + MUSCL + SSP-RK2, CFL 0.45, t = 0.1", U))
    p = O.Problem(dim=1, n=(48,), eq="swe", flux="roe", recon="eno2", integrator="ssprk3",
                  bc=("transmissive",))
    U, *_ = O.evolve(p, fi.swe_dam_break_1d(48), 0.02, 0.4)
    out.append(("swe_dam_break_roe_eno2_48", "shallow-water dam break, 48 cells, Roe + ENO2 + SSP-RK3, CFL 0.4, t = 0.02", U))
    p = O.Problem(dim=1, n=(40,), eq="mhd", flux="hll", recon="muscl_minmod", integrator="ssprk2",
                  bc=("transmissive",), gamma=2.0)
    U, *_ = O.evolve(p, fi.brio_wu_state(40), 0.05, 0.5)
    out.append(("brio_wu_hll_muscl_40", "Brio-Wu, 40 cells, gamma 2, HLL + MUSCL + SSP-RK2, CFL 0.5, t = 0.05", U))
    rng = np.random.default_rng(5)
    u0 = rng.normal(size=(1, 1, 1, 1, 40))
    p = O.Problem(dim=1, n=(40,), eq="burgers", flux="ec4", integrator="ssprk3")
    U, *_ = O.evolve(p, u0, 10.0, 0.3, max_steps=10)
    out.append(("burgers_ec4_40", "Burgers, 40 periodic cells, normal(seed 5) data, fourth-order EC flux + SSP-RK3, 10 steps, CFL 0.3", U))
    return [(n, d, np.ascontiguousarray(v, dtype=np.float64).ravel()) for n, d, v in out]


def main():
    for name, desc, vals in cases():
        with open(os.path.join(HERE, name + ".txt"), "w") as fh:
            fh.write(f"# {desc}\n# written by tests/golden/make_golden.py from the oracle; one value per line (float.hex)\n")
            for v in vals:
                fh.write(float(v).hex() + "\n")


if __name__ == "__main__":
    main()
