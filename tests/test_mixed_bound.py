"""Where the mixed-precision Newton/IP bound comes from (CPU, oracle only).

The tanh benchmark (n = 4, m = 1, T = 1024, six barrier levels of ten Newton
iterations) is unstable and saturating: at small barrier weights the iterates
sit within 1e-7 of the control box, and whether a candidate u + du is feasible
is decided at rounding level.  The final cost of the 60-iteration run is
therefore determined by the data only up to the spread that perturbations of
the size of FP32 rounding in the LQ steps produce.  These tests pin the
Python composition of the oracle's iteration against the oracle's C loop and
measure that spread; test_gpu_mixed.py asserts the mixed path against the
bound derived from it (perturbed_newton.MIXED_NEWTON_BOUND).
"""
import numpy as np

import oracle
import perturbed_newton as PN
from paper_2409_20027_amd import workloads as W

ARGS = (W.NMPC_MU_LEVELS, W.NMPC_ITERS_PER_LEVEL, W.NMPC_ALPHA0, W.NMPC_NU0)


def test_composed_iteration_reproduces_the_oracle_loop():
    p = W.nmpc_problem(seed=1, T=1024)
    ref = oracle.nmpc_solve(p, *ARGS)
    got = PN.run(p, *ARGS)
    assert np.array_equal(got["accepted"], ref["accept"])
    assert np.max(np.abs(got["cost"] - ref["cost"]) / np.abs(ref["cost"])) <= 1e-12
    assert np.max(np.abs(got["u"] - ref["u"])) <= 1e-12


def test_fp32_sized_perturbations_spread():
    """24 runs with every LQ step's data perturbed by relative 2^-24: the final
    costs spread beyond the proposed 1e-5 (so that bound cannot hold for an
    FP32 path) and stay within MIXED_NEWTON_BOUND; every first flipped
    decision sits where the unperturbed candidate is within 1e-6 of the box."""
    p = W.nmpc_problem(seed=1, T=1024)
    ref = PN.run(p, *ARGS)
    spread, firsts = [], []
    for s in range(24):
        r = PN.run(p, *ARGS, eps=PN.FP32_EPS, seed=100 + s)
        spread.append(abs(r["cost"][-1] - ref["cost"][-1]) / abs(ref["cost"][-1]))
        flips = np.nonzero(r["accepted"] != ref["accepted"])[0]
        if len(flips):
            firsts.append(int(flips[0]))
            assert ref["margin"][flips[0]] < 1e-6, (s, flips[0], ref["margin"][flips[0]])
    spread = np.array(spread)
    print(f"final-cost spread: max {spread.max():.2e}, median {np.median(spread):.2e}, first flips {sorted(set(firsts))}")
    assert 1e-5 < spread.max() <= PN.MIXED_NEWTON_BOUND
