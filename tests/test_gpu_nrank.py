"""Numerical rank without pivoting or orthogonalization (Proto-Algorithm B.1, Remarks B.2 /
B.4) through genp_numerical_rank, against the oracle."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import nrank as onr  # noqa: E402
from paper_1212_4560_amd import genp, workloads as wl  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

U64 = 2.0 ** -53


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("q,lo,hi", [(1, 0, 40), (8, 0, 40), (17, 3, 40), (32, 0, 64), (40, 0, 40), (0, 0, 16)])
def test_rank_against_the_oracle(q, lo, hi):
    """Exact-rank and Table 7.2 (tail 1e-10) matrices: the library's rank equals the oracle's
    (both COND forms) and q; at most ceil(log2(hi - lo + 1)) tests; the returned basis is
    A^T G_rank (within 4 m u |A^T| |G|); the kappa estimates match the oracle's Lanczos
    estimates on the same blocks where both are finite and below 1e7."""
    n = 96
    g = np.random.default_rng(q + 100)
    mats = [np.zeros((n + 20, n))] if q == 0 else [g.standard_normal((n + 20, q)) @ g.standard_normal((q, n)),
                                                    wl.svd_head_matrix(n, q, seed=q)[0]]
    for A in mats:
        G = g.standard_normal((A.shape[0], hi))
        o = onr.numerical_rank(A, G, lo, hi, 1e6)
        ol = onr.numerical_rank(A, G, lo, hi, 1e6, cond="lanczos")
        r = genp.numerical_rank(dev(A), dev(G), lo, hi, 1e6)
        info = r["info"]
        assert r["rank"] == o.rank == ol.rank == q
        assert info["tests"] == len(o.tests) <= math.ceil(math.log2(hi - lo + 1))
        B = host(r["B"])
        Bo = A.T @ G[:, :q]
        assert np.all(np.abs(B - Bo) <= 4 * A.shape[0] * U64 * (np.abs(A.T) @ np.abs(G[:, :q])) + 1e-300)
        kr = [k for s_, k, ok in ol.tests if s_ == q]
        if kr and math.isfinite(kr[0]) and kr[0] < 1e7:
            assert abs(info["cond_at_rank"] - kr[0]) <= 1e-6 * kr[0]


def test_argument_errors():
    A = dev(np.ones((10, 8)))
    G = dev(np.ones((10, 8)))
    for lo, hi in ((3, 3), (-1, 4), (0, 9)):
        with pytest.raises(genp.GenpError) as e:
            genp.numerical_rank(A, G[:, :max(hi, 1)] if hi <= 8 else dev(np.ones((10, hi))), lo, hi)
        assert e.value.status == genp.EINVAL


def test_fullsize_n16384():
    """m = n = 16384, A = X Y^T + E of numerical rank 16, range [0, 64]: rank 16, basis sampled
    against the host's dot products."""
    n, q, k = 16384, 16, 64
    print("nrank n=16384: inputs", flush=True)
    A, G = wl.lowrank_plus_noise(n, n, q, k, device="cuda")
    r = genp.numerical_rank(A, G, 0, k, 1e6)
    info = r["info"]
    print(f"  rank {r['rank']} tests {info['tests']} cond {info['cond_at_rank']:.3g} / {info['cond_above']:.3g}; "
          f"ms {info['ms_total']:.2f} (sketch {info['ms_sketch']:.2f}, gram {info['ms_gram']:.2f}, "
          f"search {info['ms_search']:.2f})", flush=True)
    assert r["rank"] == q and info["tests"] <= 7
    g = np.random.default_rng(3)
    J = g.integers(0, n, 32)
    C = g.integers(0, q, 32)
    B = host(r["B"])
    Gh = host(G)
    for j, c in zip(J, C):
        col = host(A[:, int(j)])
        exact = col @ Gh[:, c]
        assert abs(B[j, c] - exact) <= 4 * n * U64 * (np.abs(col) @ np.abs(Gh[:, c]))
