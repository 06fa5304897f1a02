"""Parity of the CSR path and of lambda lanes with the FP64 oracle (MI355X)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import reference as R  # noqa: E402
from workloads import sparse_zipf_logreg  # noqa: E402


@pytest.fixture(scope="module")
def cg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_18463_amd as cg
    cg._lib.load()
    return cg


def _dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.to("cuda") if dtype is None else t.to(device="cuda", dtype=dtype)


def _csr(cg, p):
    return cg.csr_matrix(_dev(p.row_ptr), _dev(p.col_idx), _dev(p.values), p.n)


@pytest.fixture(scope="module")
def small():
    return sparse_zipf_logreg(6000, 3000, 11, nnz_mean=20.0)


@pytest.mark.parametrize("b,s", [(16, 4), (32, 8), (8, 1), (4, 13)])
def test_sparse_fit_matches_oracle(cg, small, b, s):
    p = small
    X = _csr(cg, p)
    y = _dev(p.y)
    x = torch.zeros(p.n, device="cuda")
    H = 60
    ws = cg.casgd_sparse_prepare(X, b, s)
    cg.casgd_fit(X, y, x, 2.0, 1e-3, b, s, 5, 0, H, ws=ws)
    cg.casgd_check(ws)
    xo = R.casgd_csr(p.row_ptr, p.col_idx, p.values, p.n, p.y, np.zeros(p.n), 2.0, 1e-3, b, s,
                     5, 0, H)
    xg = x.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(xg - xo) / np.linalg.norm(xo) < 1e-4


def test_lanes_match_oracle_and_solo_runs(cg, small):
    p = small
    X = _csr(cg, p)
    y = _dev(p.y)
    lams = [0.0, 1e-4, 3e-3, 1e-2, 5e-2]
    L, b, s, H = len(lams), 16, 8, 40
    xl = torch.zeros(p.n, L, device="cuda")
    ws = cg.casgd_sparse_prepare(X, b, s, L)
    cg.casgd_fit_path(X, y, xl, lams, 1.5, b, s, 9, 0, H, ws=ws)
    cg.casgd_check(ws)
    got = xl.cpu().numpy().astype(np.float64)
    for l, lam in enumerate(lams):
        xo = R.casgd_csr(p.row_ptr, p.col_idx, p.values, p.n, p.y, np.zeros(p.n), 1.5, lam, b,
                         s, 9, 0, H)
        assert np.linalg.norm(got[:, l] - xo) / np.linalg.norm(xo) < 1e-4, l
        solo = torch.zeros(p.n, 1, device="cuda")
        cg.casgd_fit_path(X, y, solo, [lam], 1.5, b, s, 9, 0, H, ws=ws)
        assert torch.equal(solo[:, 0], xl[:, l]), l


@pytest.mark.parametrize("K", [1, 2, 8, 32])
def test_recurrence_split_matches_oracle(cg, small, K):
    """The lane-group recurrence split over K workgroups (rows of each block
    divided among them, deltas exchanged between steps): every split matches
    the oracle, and the unsplit form to rounding."""
    p = small
    X = _csr(cg, p)
    y = _dev(p.y)
    lams = [0.0, 1e-4, 3e-3, 1e-2, 5e-2]
    L, b, s, H = len(lams), 32, 8, 30
    ws = cg.casgd_sparse_prepare(X, b, s, L)
    out = {}
    for k in sorted({1, K}):
        xl = torch.zeros(p.n, L, device="cuda")
        cg.casgd_fit_path(X, y, xl, lams, 1.5, b, s, 9, 0, H, opts=cg.opts(rec_split=k), ws=ws)
        cg.casgd_check(ws)
        out[k] = xl.cpu().numpy().astype(np.float64)
    for l in (0, 4):
        xo = R.casgd_csr(p.row_ptr, p.col_idx, p.values, p.n, p.y, np.zeros(p.n), 1.5, lams[l],
                         b, s, 9, 0, H)
        assert np.linalg.norm(out[K][:, l] - xo) / np.linalg.norm(xo) < 1e-4, l
    assert np.linalg.norm(out[K] - out[1]) / np.linalg.norm(out[1]) < 1e-6


def test_recurrence_split_rejects_bad_values(cg, small):
    p = small
    X = _csr(cg, p)
    y = _dev(p.y)
    ws = cg.casgd_sparse_prepare(X, 32, 8, 2)
    xl = torch.zeros(p.n, 2, device="cuda")
    for k in (3, 64):
        with pytest.raises(cg.CasgdError):
            cg.casgd_fit_path(X, y, xl, [0.0, 1e-3], 1.5, 32, 8, 9, 0, 1,
                              opts=cg.opts(rec_split=k), ws=ws)


@pytest.mark.parametrize("L,m,nnz", [(40, 4000, 20.0), (4, 20000, 8.0)])
def test_tail_update_one_column_per_wave(cg, L, m, nnz):
    """The tail update's whole-wave form (more than 32 lanes; or a head panel
    of 128 columns, which leaves room for one scratch list per wave: few
    columns are frequent enough per block when m is large and rows short)
    against the oracle."""
    p = sparse_zipf_logreg(m, 3000, 13, nnz_mean=nnz)
    X = _csr(cg, p)
    y = _dev(p.y)
    lams = list(np.geomspace(1e-5, 1e-2, L))
    b, s, H = 16, 8, 30
    ws = cg.casgd_sparse_prepare(X, b, s, L)
    xl = torch.zeros(p.n, L, device="cuda")
    cg.casgd_fit_path(X, y, xl, lams, 1.5, b, s, 9, 0, H, ws=ws)
    cg.casgd_check(ws)
    got = xl.cpu().numpy().astype(np.float64)
    for l in (0, L - 1):
        xo = R.casgd_csr(p.row_ptr, p.col_idx, p.values, p.n, p.y, np.zeros(p.n), 1.5, lams[l],
                         b, s, 9, 0, H)
        assert np.linalg.norm(got[:, l] - xo) / np.linalg.norm(xo) < 1e-4, l


def test_sparse_equals_dense_on_densified(cg, small):
    p = small
    D = p.to_dense()
    n = p.n
    ld = (n + 3) // 4 * 4
    Dp = np.zeros((p.m, ld), np.float32)
    Dp[:, :n] = D
    Xd = cg.dense_matrix(_dev(Dp), n=n)
    Xs = _csr(cg, p)
    y = _dev(p.y)
    xs = torch.zeros(n, device="cuda")
    xd = torch.zeros(n, device="cuda")
    ws = cg.casgd_sparse_prepare(Xs, 16, 4)
    cg.casgd_fit(Xs, y, xs, 2.0, 1e-3, 16, 4, 3, 0, 50, ws=ws)
    cg.casgd_fit(Xd, y, xd, 2.0, 1e-3, 16, 4, 3, 0, 50)
    a, d = xs.cpu().numpy(), xd.cpu().numpy()
    assert np.linalg.norm(a - d) / np.linalg.norm(d) < 1e-5


def test_sparse_snapshots_and_resume(cg, small):
    p = small
    X = _csr(cg, p)
    y = _dev(p.y)
    L = 2
    ws = cg.casgd_sparse_prepare(X, 16, 4, L)
    hist = torch.zeros(3, p.n, L, device="cuda")
    x = torch.zeros(p.n, L, device="cuda")
    o = cg.opts(snapshot_every=4, x_history=hist)
    cg.casgd_fit_path(X, y, x, [1e-4, 1e-2], 2.0, 16, 4, 1, 0, 12, opts=o, ws=ws)
    ref = torch.zeros(p.n, L, device="cuda")
    for k in range(3):
        cg.casgd_fit_path(X, y, ref, [1e-4, 1e-2], 2.0, 16, 4, 1, 4 * k, 4, ws=ws)
        assert torch.equal(hist[k], ref)
    assert torch.equal(ref, x)


def test_c4_scale_sampled_check(cg):
    """Full-size sparse workload (10^6 x 2^17, ~50 nnz/row, 32 lambdas,
    b=128, s=16): three outer iterations, four lanes checked against the
    oracle (which only touches the sampled rows)."""
    from workloads import lambda_path_c4, sparse_c4
    p = sparse_c4(42)
    X = _csr(cg, p)
    y = _dev(p.y)
    lams = lambda_path_c4()
    L, b, s, H = len(lams), 128, 16, 3
    ws = cg.casgd_sparse_prepare(X, b, s, L)
    xl = torch.zeros(p.n, L, device="cuda")
    cg.casgd_fit_path(X, y, xl, list(lams), 8.0, b, s, 42, 0, H, ws=ws)
    cg.casgd_check(ws)
    got = xl.cpu().numpy().astype(np.float64)
    for l in (0, 10, 20, 31):
        xo = R.casgd_csr(p.row_ptr, p.col_idx, p.values, p.n, p.y, np.zeros(p.n), 8.0,
                         lams[l], b, s, 42, 0, H)
        assert np.linalg.norm(got[:, l] - xo) / np.linalg.norm(xo) < 1e-4, l
