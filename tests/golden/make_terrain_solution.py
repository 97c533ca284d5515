"""Writes the oracle's reference solution of the 32x8x16 terrain channel.

The workload: terrain-following channel of 32 x 8 x 16 cells (Gaussian ridge,
geometry degree 4), DG Q4, isothermal background coefficients, penalty 2, the
right-hand side of ``synth_inputs.rhs_terrain(0)`` evaluated at the oracle's
own dof coordinates and used as the coefficient vector b.  The oracle's
preconditioned CG (with its separable cell blocks) runs to a 1e-13 relative
residual.  Only ``oracle/`` and ``synth_inputs/`` are called.

Output: ``terrain32x8x16_k4_rhs0_solution.npy`` (float64, 512,000 values) and
``terrain32x8x16_k4_rhs0_solution.txt`` (iterations, residuals, wall time).

    python tests/golden/make_terrain_solution.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth_inputs as si  # noqa: E402

NAME = "terrain32x8x16_k4_rhs0_solution"


def main():
    m = si.terrain_mesh(32, 8, 16, g=4)
    p = oracle.Problem(m, 4)
    p.set_coefficient_functions(*si.terrain_coefficients())
    b = si.rhs_terrain(0)(*p.dof_coords())
    t0 = time.time()
    x, info = oracle.solvers.cg(p.apply, b, precond=p.bj_apply, rtol=1e-13, max_iter=5000)
    dt = time.time() - t0
    assert info.converged, info.true_rel_res
    np.save(os.path.join(HERE, NAME + ".npy"), x)
    hist = np.array(info.history)
    it8 = int(np.argmax(hist <= 1e-8))
    with open(os.path.join(HERE, NAME + ".txt"), "w") as f:
        f.write(f"# oracle CG + separable block Jacobi, 32x8x16 terrain channel, Q4, rhs_terrain(0)\n")
        f.write(f"iterations {info.iters}\n")
        f.write(f"iterations_to_1e-8 {it8}\n")
        f.write(f"true_rel_res {info.true_rel_res:.3e}\n")
        f.write(f"solution_norm {np.linalg.norm(x):.17e}\n")
        f.write(f"wall_s {dt:.1f}\n")
    print(f"{info.iters} iterations, residual {info.true_rel_res:.2e}, {dt:.0f} s")


if __name__ == "__main__":
    main()
