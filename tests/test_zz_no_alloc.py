"""The allocation-free numerical rank (genp_numerical_rank_noalloc: scratch from the library's
fixed device array, no hipMalloc) against the allocating entry point genp_numerical_rank, both
called through the C ABI on the same inputs, twice in a row with the second problem smaller.
At these sizes both take the same split-K slicing, so the sketch B must be bit-identical and the
rank, the number of COND tests and the kappa estimates equal; the rank is also the oracle's."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import nrank as onr  # noqa: E402
from paper_1212_4560_amd import genp  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def same(a, b):
    return (a == b) or (math.isnan(a) and math.isnan(b))


@pytest.mark.parametrize("order", ["noalloc_first", "alloc_first"])
def test_noalloc_matches_allocating_entry_point(order):
    cases = [(3000, 2048, 12, 48, 1), (700, 500, 5, 20, 2)]   # the second call is smaller
    for m, n, q, hi, seed in cases:
        print(f"noalloc m={m} n={n} q={q} range [0, {hi}] ({order})", flush=True)
        g = np.random.default_rng(seed)
        A = g.standard_normal((m, q)) @ g.standard_normal((q, n)) + 1e-11 * g.standard_normal((m, n))
        G = g.standard_normal((m, hi))
        Ad, Gd = dev(A), dev(G)
        outs = {}
        for kind in (("noalloc", "alloc") if order == "noalloc_first" else ("alloc", "noalloc")):
            B = torch.full((n, hi), float("nan"), dtype=torch.float64, device="cuda")
            outs[kind] = genp.numerical_rank(Ad, Gd, 0, hi, 1e6, B=B, noalloc=(kind == "noalloc"))
        r1, r2 = outs["alloc"], outs["noalloc"]
        i1, i2 = r1["info"], r2["info"]
        torch.cuda.synchronize()
        assert r2["rank"] == r1["rank"] == q == onr.numerical_rank(A, G, 0, hi, 1e6).rank
        assert i2["tests"] == i1["tests"]
        assert same(i2["cond_at_rank"], i1["cond_at_rank"]) and same(i2["cond_above"], i1["cond_above"])
        assert math.isnan(i2["ms_total"])
        assert torch.equal(r2["B"], r1["B"])
