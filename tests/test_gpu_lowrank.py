"""Randomized low-rank approximation (Proto-Algorithm 5.1, orthogonal basis of Remark 5.4)
through genp_lowrank, against the oracle and the generator's exact singular spaces."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import lowrank as ol  # noqa: E402
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


def _common_checks(A, r, oracle_res):
    m, n = A.shape
    T, W = host(r["T"]), host(r["W"])
    s = r["rank"]
    info = r["info"]
    assert s == oracle_res.rank
    assert np.allclose(T.T @ T, np.eye(s), atol=1e-13)
    assert np.all(np.abs(W - A @ T) <= 4 * n * U64 * (np.abs(A) @ np.abs(T)) + 1e-300)
    assert np.isclose(info["a_fro"], np.linalg.norm(A), rtol=1e-13)
    res_host = np.linalg.norm(A - W @ T.T)
    assert abs(info["resid_fro"] - res_host) <= 1e-6 * res_host + 64 * U64 * np.linalg.norm(A)
    perm = r["perm"]
    assert sorted(perm) == list(range(len(perm)))
    assert perm[0] == oracle_res.perm[0]
    return T, W


@pytest.mark.parametrize("n,q,extra", [(64, 1, 0), (128, 8, 5), (256, 32, 0), (256, 8, 16)])
def test_table_7_2_matrices(n, q, extra):
    """A = S diag(1/j, 1e-10) T^T: the library keeps s = q columns like the oracle, T is
    orthonormal, W = A T, the reported norms match the host's, and the projection residual
    is of order sigma_{q+1} (within Remark 5.2's bound with oversampling, within 1e6 sigma_{q+1}
    without; the oracle's residual for the same G is the yardstick)."""
    for seed in range(3):
        A, S, sig, Tt, G = wl.svd_head_matrix(n, q, seed=seed, rho_plus=q + extra)
        o = ol.lowrank(A, G, 1e-8, 1e-4)
        r = genp.lowrank(dev(A), q + extra, G=dev(G), tau=1e-8, tau2=1e-4)
        T, W = _common_checks(A, r, o)
        res2 = np.linalg.norm(A - W @ T.T, 2)
        bound = (1 + 9 * np.sqrt((q + extra) * n)) * sig[q] if extra else 1e6 * sig[q]
        assert res2 <= max(bound, 10 * ol.projection_residual(A, o.T))
        assert not r["info"]["failed"]


@pytest.mark.parametrize("n,q", [(64, 8), (256, 32)])
def test_table_7_3_toeplitz_multiplier(n, q):
    """The same with a random Toeplitz multiplier (m + rho_+ - 1 parameters)."""
    A, S, sig, Tt, p = wl.svd_head_matrix(n, q, seed=7, mult=wl.MULT_TOEPLITZ, rho_plus=q + 4)
    G = ol.toeplitz_rect(p, n, q + 4)
    o = ol.lowrank(A, G, 1e-8, 1e-4)
    r = genp.lowrank(dev(A), q + 4, p=dev(p), tau=1e-8, tau2=1e-4)
    T, W = _common_checks(A, r, o)
    assert np.linalg.norm(A - W @ T.T, 2) <= (1 + 9 * np.sqrt((q + 4) * n)) * sig[q]


def test_rectangular_exact_rank_and_ahat():
    """m != n, A of exact rank 5, rho_+ = 12: s = 5, residual at the rounding level, A_hat =
    W T^T stored when asked for."""
    m, n = 300, 200
    g = np.random.default_rng(5)
    A = g.standard_normal((m, 5)) @ g.standard_normal((5, n))
    G = g.standard_normal((m, 12))
    o = ol.lowrank(A, G, 1e-10, 1e-10)
    r = genp.lowrank(dev(A), 12, G=dev(G), tau=1e-10, tau2=1e-10, want_ahat=True)
    T, W = _common_checks(A, r, o)
    assert r["rank"] == 5 and not r["info"]["failed"]
    assert r["info"]["resid_fro"] <= 1e-13 * r["info"]["a_fro"]
    assert np.allclose(host(r["Ahat"]), W @ T.T, atol=1e-13 * np.abs(A).max())


def test_failure_and_argument_errors():
    A, S, sig, Tt, G = wl.svd_head_matrix(64, 8, seed=2)
    r = genp.lowrank(dev(A), 8, G=dev(G), tau=1e-8, tau2=1e-30)
    assert r["info"]["failed"] == 1
    r = genp.lowrank(dev(A), 8, G=dev(G), tau=10.0, tau2=1e-4)   # no column kept
    assert r["rank"] == 0 and r["info"]["failed"] == 1
    Gbig = dev(np.random.default_rng(1).standard_normal((64, 65)))
    with pytest.raises(genp.GenpError) as e:
        genp.lowrank(dev(A), 65, G=Gbig)
    assert e.value.status == genp.EINVAL


def test_rank_one_multiplier():
    A, S, sig, Tt, G = wl.svd_head_matrix(64, 1, seed=4)
    o = ol.lowrank(A, G, 1e-8, 1e-4)
    r = genp.lowrank(dev(A), 1, G=dev(G), tau=1e-8, tau2=1e-4)
    _common_checks(A, r, o)
    assert r["rank"] == 1


def test_fullsize_n16384():
    """m = n = 16384, A = X Y^T + N with X, Y Gaussian of 16 columns and ||N|| ~ 1e-10 relative,
    rho_+ = 32: s = 16 like the oracle on the same A and G; T orthonormal; 64 sampled entries
    of W against the host's dot products; the residual within a factor 2 of the oracle's (both
    project on the first 16 pivoted columns of the sketch, whose noise tilts the subspace, so
    the residual is a few times ||N||_F rather than ||N||_F)."""
    n, q, k = 16384, 16, 32
    print("lowrank n=16384: inputs", flush=True)
    g = np.random.default_rng(11)
    X = torch.from_numpy(g.standard_normal((n, q))).cuda()
    Y = torch.from_numpy(g.standard_normal((n, q))).cuda()
    A = X @ Y.T
    scale = 1e-10 * float(torch.linalg.norm(A)) / n
    Nn = torch.from_numpy(g.standard_normal((n, n))).cuda() * scale
    A += Nn
    nfro = float(torch.linalg.norm(Nn))
    del Nn
    G = torch.from_numpy(g.standard_normal((n, k))).cuda()
    r = genp.lowrank(A, k, G=G, tau=1e-8, tau2=1e-6)
    info = r["info"]
    print(f"  rank {r['rank']}, ms {info['ms_total']:.2f} (sketch {info['ms_sketch']:.2f}, basis "
          f"{info['ms_basis']:.2f}, project {info['ms_project']:.2f}, resid {info['ms_resid']:.2f})", flush=True)
    assert r["rank"] == q and not info["failed"]
    assert np.isclose(info["a_fro"], float(torch.linalg.norm(A)), rtol=1e-12)
    T = host(r["T"])
    assert np.allclose(T.T @ T, np.eye(q), atol=1e-13)
    I = g.integers(0, n, 64)
    J = g.integers(0, q, 64)
    Ah = host(A[torch.as_tensor(I, device="cuda")])
    W = host(r["W"])
    for t, (i, j) in enumerate(zip(I, J)):
        exact = Ah[t] @ T[:, j]
        assert abs(W[i, j] - exact) <= 4 * n * U64 * (np.abs(Ah[t]) @ np.abs(T[:, j]))
    print("  oracle on the host", flush=True)
    o = ol.lowrank(host(A), host(G), 1e-8, 1e-6)
    print(f"  resid {info['resid_fro']:.3e} oracle {o.resid_fro:.3e} ||N||_F {nfro:.3e}", flush=True)
    assert o.rank == q
    assert 0.5 * o.resid_fro <= info["resid_fro"] <= 2.0 * o.resid_fro
    assert info["resid_fro"] >= 0.5 * nfro
