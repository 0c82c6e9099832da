"""Write the oracle's gradient of a long march as a compact text fixture.

    python tests/golden/make_oracle_gradients.py NX NY T

writes tests/golden/oracle_gradient_<NX>x<NY>_T<T>.txt.  The gradient is
dR/d(u0, v0) of R = KE(T)/KE(0) (Eq. 10's ratio with the time steps of the
forward run held fixed, Sec. 3.4) from the oracle's reverse-mode AD through
the whole march, for the Gaussian seed 0 at RMS 1e-3 of the benchmark
physics.  A whole field is too large to keep, so the file holds what a test
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
from paper_2608_04085_amd.config import RTConfig  # noqa: E402

DIRECTION_SEEDS = list(range(5000, 5008))


def fixture_name(nx, ny, T):
    return os.path.join(HERE, f"oracle_gradient_{nx}x{ny}_T{T:g}.txt")


def main():
    nx, ny, T = int(sys.argv[1]), int(sys.argv[2]), float(sys.argv[3])
    cfg = RTConfig(nx=nx, ny=ny)
    uv = inputs.seed_batch(cfg, [0], rms=1e-3)
    t0 = time.time()
    R, g, n, _ = Oracle.from_config(cfg).grad_u0(uv, T)
    el = time.time() - t0
    delta = float(np.sqrt(np.sum(uv * uv) * cfg.dx * cfg.dy))
    gd = [float(np.sum(g * inputs.direction_batch(cfg, [s], delta))) for s in DIRECTION_SEEDS]
    flat = g.ravel()
    top = np.argsort(-np.abs(flat), kind="stable")[:32]
    rnd = np.random.default_rng(123).choice(flat.size, size=32, replace=False)
    idx = np.concatenate([top, rnd])
    with open(fixture_name(nx, ny, T), "w") as f:
        f.write("# Oracle gradient of R = KE(T)/KE(0), frozen time steps, reverse-mode AD through the march.\n")
        f.write(f"# Written by tests/golden/make_oracle_gradients.py {nx} {ny} {T:g} ({el:.0f} s).\n")
        f.write("# Benchmark physics (RTConfig defaults), Gaussian seed 0 scaled to RMS 1e-3.\n")
        f.write("# gd: inner products with inputs.direction_batch(cfg, [s], delta) for s in dir_seeds,\n")
        f.write("# delta the seed's velocity L2 norm; idx: flat indices into [1][2][ny][nx]; gval: g there.\n")
        f.write(f"nx {nx}\nny {ny}\nT {T!r}\nnsteps {int(n[0])}\n")
        f.write(f"R {float(R[0])!r}\n")
        f.write(f"gnorm {float(np.linalg.norm(flat))!r}\n")
        f.write(f"gmax {float(np.max(np.abs(flat)))!r}\n")
        f.write("dir_seeds " + " ".join(str(s) for s in DIRECTION_SEEDS) + "\n")
        f.write("gd " + " ".join(repr(x) for x in gd) + "\n")
        f.write("idx " + " ".join(str(int(i)) for i in idx) + "\n")
        f.write("gval " + " ".join(repr(float(flat[i])) for i in idx) + "\n")
    print(f"{nx}x{ny} T={T:g}: {int(n[0])} steps, R {float(R[0])!r}, {el:.0f} s -> {fixture_name(nx, ny, T)}")


if __name__ == "__main__":
    main()
