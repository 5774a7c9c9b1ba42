"""GPU test of fem_lcp_noalloc, the allocation-free variant of fem_lcp: caller-owned device
buffers and the library's fixed device workspace give the same results as fem_lcp, on calls
in a row whose second input is smaller than the first (the workspace keeps the last call's
contents, which must not leak into the next)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _problem(m, q_shift, seed):
    """W = M M^T / k + I/2 (symmetric positive definite) and q ~ N(q_shift, 1)."""
    rng = np.random.default_rng([m, seed, 7])
    k = m + 8
    M = rng.normal(size=(m, k))
    W = M @ M.T / k + 0.5 * np.eye(m)
    q = rng.normal(size=m) + q_shift
    return W, q


def _noalloc(W, q, stream=None):
    import torch
    from paper_2503_06922_amd import fem
    Wd = torch.tensor(np.ascontiguousarray(W.T), dtype=torch.float64, device="cuda")
    qd = torch.tensor(q, dtype=torch.float64, device="cuda")
    yd = torch.full((q.shape[0],), np.nan, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    path = fem.fem_lcp_noalloc(Wd, qd, yd, stream)
    return yd.cpu().numpy(), path


def test_noalloc_lcp_matches_fem_lcp_on_calls_in_a_row():
    import torch
    from paper_2503_06922_amd import fem
    cases = [
        _problem(400, -0.2, 0),                   # active set beyond 128: HBM-factor workspace
        (lambda W: (W, -W @ np.full(150, 0.25)))(_problem(150, 0.0, 1)[0]),  # all 150 active
        _problem(90, 0.3, 2),                     # factor in LDS
        _problem(40, 0.0, 3),                     # LDS active set
        _problem(300, -0.3, 4),                   # the workspace again after smaller calls
    ]
    expect_path = [2, 2, 1, 0, 2]
    side = torch.cuda.Stream()
    for i, (W, q) in enumerate(cases):
        y_ref, p_ref = fem.fem_lcp(W, q)
        y, p = _noalloc(W, q, side if i % 2 else None)
        print("case", i, "m", q.shape[0], "path", p, "active", int(np.sum(y > 0)))
        assert p == p_ref == expect_path[i], (i, p, p_ref)
        assert np.array_equal(y, y_ref), (i, np.abs(y - y_ref).max())


def test_noalloc_lcp_rejects_sizes_beyond_its_workspace():
    import torch
    from paper_2503_06922_amd import fem
    m = fem.FEM_LCP_NOALLOC_MAX_M + 1
    Wd = torch.eye(m, dtype=torch.float64, device="cuda")
    qd = torch.zeros(m, dtype=torch.float64, device="cuda")
    yd = torch.zeros(m, dtype=torch.float64, device="cuda")
    with pytest.raises(fem.FemError) as e:
        fem.fem_lcp_noalloc(Wd, qd, yd)
    assert e.value.status == fem.FEM_E_INVAL
    # the largest accepted size still runs
    W, q = _problem(fem.FEM_LCP_NOALLOC_MAX_M, -0.1, 5)
    y_ref, p_ref = fem.fem_lcp(W, q)
    y, p = _noalloc(W, q)
    assert p == p_ref and np.array_equal(y, y_ref)
