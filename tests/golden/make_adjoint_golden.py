"""Write the gradient oracle's values for the differentiated Kelvin--Helmholtz run at its full
shape (run from the repository root: python tests/golden/make_adjoint_golden.py; about five
minutes on 8 cores). The run: 2D Euler on the periodic unit square at 256^2, samples 0 and 1
of seed 1915 (c_k, phi_k as the input builder draws them), MUSCL-minmod + Rusanov + SSP-RK3,
500 steps of the fixed dt = 0.4 / M_0 (M_0 the maximum wave speed of sample 0's initial
state), Q = the kinetic energy of the rows |y_j - 0.5| < 0.1. Every value comes from the
oracle alone (oracle/adjoint_torch.py, autograd in float64 on the CPU) on inputs from
fv_inputs; the GPU adjoint test compares with them. Output: adjoint_kh256_500.txt, lines
"Q <hex>" and "g <k> <hex>" per sample."""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import fv_inputs as fi  # noqa: E402
import oracle as O  # noqa: E402
from oracle import adjoint_torch as AT  # noqa: E402

N, STEPS, SEED, SAMPLES, CFL = 256, 500, 1915, (0, 1), 0.4
OUT = os.path.join(HERE, "adjoint_kh256_500.txt")


def timestep():
    c, phi = fi.kh_coefficients(SEED, [0])
    U0 = fi.kh2d_state(N, c, phi)
    p = O.Problem(dim=2, n=(N, N), eq="euler", flux="rusanov", recon="muscl_minmod",
                  integrator="ssprk3")
    M, _ = O.max_speed(p, U0[0])
    return CFL / M


def main():
    dt = timestep()
    c, phi = fi.kh_coefficients(SEED, list(SAMPLES))
    U0 = fi.kh2d_state(N, c, phi)
    t0 = time.time()
    Q, gc, gp = AT.qoi_and_gradient(c, phi, N, dt, STEPS, U0_values=U0)
    g = np.concatenate([gc, gp], axis=1)
    with open(OUT, "w") as fh:
        fh.write(f"# gradient oracle, KH {N}^2, seed {SEED}, samples {list(SAMPLES)}, "
                 f"{STEPS} steps of dt = {dt.hex()} (CFL {CFL} of sample 0's initial state), "
                 "MUSCL-minmod + Rusanov + SSP-RK3; band |y - 0.5| < 0.1\n")
        for b in range(len(SAMPLES)):
            fh.write(f"sample {SAMPLES[b]}\n")
            fh.write(f"Q {float(Q[b]).hex()}\n")
            for k in range(g.shape[1]):
                fh.write(f"g {k} {float(g[b, k]).hex()}\n")
    print(f"wrote {OUT} in {time.time() - t0:.0f} s")


def load(path=OUT):
    """(dt, {sample: (Q, g[20])}) from the fixture."""
    dt, out, cur = None, {}, None
    for line in open(path):
        if line.startswith("#"):
            dt = float.fromhex(line.split("dt = ")[1].split()[0])
            continue
        f = line.split()
        if f[0] == "sample":
            cur = int(f[1])
            out[cur] = [None, np.zeros(20)]
        elif f[0] == "Q":
            out[cur][0] = float.fromhex(f[1])
        elif f[0] == "g":
            out[cur][1][int(f[1])] = float.fromhex(f[2])
    return dt, {k: (v[0], v[1]) for k, v in out.items()}


if __name__ == "__main__":
    main()
