"""Seeded random cross-checks of the whole product path against the CPU oracle: random
shapes (log-uniform in [8, 5000], one in five in [1000, 6000]), densities, strides and modes under random schedules
(any base kernel and tile variant, Strassen-Winograd cutoff, odd-size rule, k split, M4RM table width and
workspace plan).
Every result must be bit-exact whatever the schedule."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from gf2_testutil import run_and_check


@pytest.fixture(scope="module")
def g():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0811_1714_amd as g
    g.lib()
    return g


def random_case(rng, g):
    m, k, n = (int(x) for x in np.exp(rng.uniform(np.log(8), np.log(5000), 3)))
    u = rng.uniform()
    kernel = g.KERNEL_M4RM if u < 0.7 else (g.KERNEL_MFMA if u < 0.85 else g.KERNEL_CUBIC)
    variant = int(rng.integers(g.kernel_variants(kernel))) if kernel == g.KERNEL_M4RM else 0
    # Cutoffs from min(m, k, n) / 1.4 down to / 8 (one to three levels), at least 64.
    cutoff = 0 if rng.uniform() < 0.4 else max(64, int(min(m, k, n) / 2 ** rng.uniform(0.5, 3)))
    splitk = 1 if rng.uniform() < 0.6 else int(rng.integers(2, 9))
    odd = int(rng.integers(2)) if cutoff else 0
    c = dict(m=m, k=k, n=n, accumulate=bool(rng.integers(2)), p=float(rng.choice([0.5, 0.1, 0.01])),
             lda_pad=int(rng.integers(3)), ldb_pad=int(rng.integers(3)), ldc_pad=int(rng.integers(3)))
    # Table width: 8, or 4..7 on the tiles that offer narrow tables.
    kappa = int(rng.choice([0, 4, 5, 6, 7])) if kernel == g.KERNEL_M4RM and variant in NARROW else 0
    # Workspace plan: breadth-first, or two temporaries at the top level (where it applies).
    memory = int(rng.integers(2)) if cutoff else 0
    c["schedule"] = (kernel, variant, cutoff, splitk, odd, kappa, memory)
    return c


NARROW = (1, 2, 3, 4, 12, 13, 18, 19, 20)   # tiles with tables of 4..7 bits


def case(i, g):
    """Case i: its own generator; one case in five has all three dimensions in [1000, 6000]."""
    rng = np.random.default_rng(500000 + i)
    c = random_case(rng, g)
    if rng.uniform() < 0.2:
        c["m"], c["k"], c["n"] = (int(x) for x in np.exp(rng.uniform(np.log(1000), np.log(6000), 3)))
        if c["schedule"][2]:
            s = list(c["schedule"])
            s[2] = max(64, int(min(c["m"], c["k"], c["n"]) / 2 ** rng.uniform(0.5, 3)))
            c["schedule"] = tuple(s)
    return c


@pytest.mark.parametrize("block", range(8))
def test_random_shapes_and_schedules(g, block):
    for i in range(32 * block, 32 * block + 32):
        c = case(i, g)
        print(f"case {i}: {c}", flush=True)
        run_and_check(g, c["m"], c["k"], c["n"], schedule=g.Schedule(*c["schedule"]), accumulate=c["accumulate"],
                      p=c["p"], seed=500000 + i, lda_pad=c["lda_pad"], ldb_pad=c["ldb_pad"], ldc_pad=c["ldc_pad"])
