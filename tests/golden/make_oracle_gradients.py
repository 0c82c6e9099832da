"""Write the oracle's gradient of a long march as a compact text fixture.

    python tests/golden/make_oracle_gradients.py NX NY T
    python tests/golden/make_oracle_gradients.py J N T

The first form writes tests/golden/oracle_gradient_<NX>x<NY>_T<T>.txt: the
gradient dR/d(u0, v0) of R = KE(T)/KE(0) (Eq. 10's ratio with the time
steps of the forward run held fixed, Sec. 3.4) from the oracle's
reverse-mode AD through the whole march, for the Gaussian seed 0 at RMS
1e-3 of the benchmark physics.  The second writes
oracle_gradient_J_paper<N>_T<T>.txt: the gradient of the paper's objective
J of Eq. 8 against the oracle's unperturbed run, on the paper's physics at
N x N (u_y only), for the same seed.  A whole field is too large to keep, so the file holds what a test
can compare without it: the step count, R, the Euclidean norm and the
largest entry of the gradient, its inner products with eight seeded
directions, and its entries at 32 cells where it is largest plus 32 seeded
cells.  Only the oracle and the seeded input generators are called.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.rto import Oracle  # noqa: E402
from paper_2608_04085_amd import inputs  # noqa: E402
from paper_2608_04085_amd.config import RTConfig, paper_preset  # noqa: E402

DIRECTION_SEEDS = list(range(5000, 5008))


def fixture_name(nx, ny, T, objective="R"):
    if objective == "J":
        return os.path.join(HERE, f"oracle_gradient_J_paper{nx}_T{T:g}.txt")
    return os.path.join(HERE, f"oracle_gradient_{nx}x{ny}_T{T:g}.txt")


def main():
    objective = "J" if sys.argv[1] == "J" else "R"
    if objective == "J":
        n, T = int(sys.argv[2]), float(sys.argv[3])
        cfg = paper_preset(n)
        nx = ny = n
    else:
        nx, ny, T = int(sys.argv[1]), int(sys.argv[2]), float(sys.argv[3])
        cfg = RTConfig(nx=nx, ny=ny)
    o = Oracle.from_config(cfg)
    uv = inputs.seed_batch(cfg, [0], rms=1e-3)
    t0 = time.time()
    if objective == "J":
        R, g, nsteps, _ = o.grad_ek_anomaly(uv, T, o.baseline_ek(T))
        what = "J of Eq. 8 against the oracle's unperturbed run, paper physics (paper_preset), u_y only"
    else:
        R, g, nsteps, _ = o.grad_u0(uv, T)
        what = "R = KE(T)/KE(0), benchmark physics (RTConfig defaults)"
    el = time.time() - t0
    delta = float(np.sqrt(np.sum(uv * uv) * cfg.dx * cfg.dy))
    gd = [float(np.sum(g * inputs.direction_batch(cfg, [s], delta))) for s in DIRECTION_SEEDS]
    flat = g.ravel()
    top = np.argsort(-np.abs(flat), kind="stable")[:32]
    nz = np.flatnonzero(flat)  # the masked component's entries are zero by construction
    rnd = nz[np.random.default_rng(123).choice(nz.size, size=32, replace=False)]
    idx = np.concatenate([top, rnd])
    args = " ".join(sys.argv[1:])
    with open(fixture_name(nx, ny, T, objective), "w") as f:
        f.write(f"# Oracle gradient of {what};\n")
        f.write("# frozen time steps, reverse-mode AD through the march.\n")
        f.write(f"# Written by tests/golden/make_oracle_gradients.py {args} ({el:.0f} s).\n")
        f.write("# Gaussian seed 0 (inputs.seed_batch) scaled to RMS 1e-3.\n")
        f.write("# gd: inner products with inputs.direction_batch(cfg, [s], delta) for s in dir_seeds,\n")
        f.write("# delta the seed's velocity L2 norm; idx: flat indices into [1][2][ny][nx]; gval: g there.\n")
        f.write(f"nx {nx}\nny {ny}\nT {T!r}\nnsteps {int(nsteps[0])}\n")
        f.write(f"R {float(R[0])!r}\n")
        f.write(f"gnorm {float(np.linalg.norm(flat))!r}\n")
        f.write(f"gmax {float(np.max(np.abs(flat)))!r}\n")
        f.write("dir_seeds " + " ".join(str(s) for s in DIRECTION_SEEDS) + "\n")
        f.write("gd " + " ".join(repr(x) for x in gd) + "\n")
        f.write("idx " + " ".join(str(int(i)) for i in idx) + "\n")
        f.write("gval " + " ".join(repr(float(flat[i])) for i in idx) + "\n")
    print(f"{args}: {int(nsteps[0])} steps, objective {float(R[0])!r}, {el:.0f} s -> "
          f"{fixture_name(nx, ny, T, objective)}")


if __name__ == "__main__":
    main()
