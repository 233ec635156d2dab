"""Pin of the GPU solver's iteration counts against the paper's table for the
Fichera corner with K = 448 patches (Sec. 5: PCG with one V-cycle, 1+1
smoothing, tau = 0.25, sigma = 5 h^-2, relative tolerance 1e-8), with the
library's default reading of the smoother's constants.

The constants are a reading (the paper leaves them to its references); the
default was chosen because it reproduces the table.  Asserted, for p = 2, 3,
4 and l = 1..4: every count within 20% of the paper's, and the growth under
refinement that the paper shows (the count at l = 4 at least 15% above the
count at l = 1; the paper's grow by 35% to 47%)."""
import json
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _say(msg):
    print(f"[gpu-fichera] {msg}", flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("p", [2, 3, 4])
def test_fichera_counts_match_paper_table(p):
    import torch
    from paper_1804_02539_amd import igamg, workloads as W
    assert torch.cuda.is_available()
    with open(os.path.join(GOLD, "iteration_counts.json")) as fh:
        paper = json.load(fh)["fichera_K448"]
    counts = []
    for lev in (1, 2, 3, 4):
        prob = W.fichera(p, lev + 1, split=4)
        S = igamg.Solver(prob)
        f = torch.as_tensor(S.load_vector(75.0 * np.pi ** 2, 5.0), device="cuda:0")
        _, info = S.solve(f, tol=1e-8)
        ref = paper[str(lev)][str(p)]
        _say(f"p={p} l={lev}: N={S.N}, {info.iterations} iterations (paper {ref})")
        assert info.converged and info.rel_residual <= 1e-8
        assert abs(info.iterations - ref) <= 0.2 * ref, (p, lev, info.iterations, ref)
        counts.append(info.iterations)
        del S, f
        torch.cuda.empty_cache()
    assert counts[-1] >= 1.15 * counts[0], counts
