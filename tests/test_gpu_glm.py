"""Linear and Poisson losses (Sec. 2.1 losses, Sec. 3.1 residuals) on the GPU
paths other than the dense fit (checked per outer iteration in
test_gpu_fused_local.py): the CSR path and its lambda lanes, the batched
launch, and the loss evaluation, each against the FP64 oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import reference as R  # noqa: E402
from workloads import dense_glm, sparse_zipf_glm  # noqa: E402

ETA_CSR = {"logistic": 2.0, "linear": 0.5, "poisson": 0.25}


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


@pytest.fixture(scope="module")
def sparse():
    return {loss: sparse_zipf_glm(6000, 3000, 23, loss, nnz_mean=20.0)
            for loss in ("linear", "poisson")}


@pytest.mark.parametrize("loss", ["linear", "poisson"])
@pytest.mark.parametrize("b,s", [(16, 4), (32, 8), (4, 13)])
def test_csr_fit_and_lanes_match_oracle(cg, sparse, loss, b, s):
    p = sparse[loss]
    X = cg.csr_matrix(_dev(p.row_ptr), _dev(p.col_idx), _dev(p.values), p.n)
    y = _dev(p.y)
    lams = [0.0, 1e-3, 3e-2]
    eta, H = ETA_CSR[loss], 40
    xl = torch.zeros(p.n, len(lams), device="cuda")
    ws = cg.casgd_sparse_prepare(X, b, s, len(lams))
    cg.casgd_fit_path(X, y, xl, lams, eta, b, s, 3, 0, H, opts=cg.opts(loss=loss), ws=ws)
    cg.casgd_check(ws)
    got = xl.cpu().numpy().astype(np.float64)
    for l, lam in enumerate(lams):
        xo = R.casgd_csr(p.row_ptr, p.col_idx, p.values, p.n, p.y, np.zeros(p.n), eta, lam, b, s,
                         3, 0, H, loss=loss)
        rel = np.linalg.norm(got[:, l] - xo) / np.linalg.norm(xo)
        assert rel < 1e-4, (l, rel)
    # single-lane fit through casgd_fit equals lane 0 bitwise
    x1 = torch.zeros(p.n, device="cuda")
    cg.casgd_fit(X, y, x1, eta, lams[0], b, s, 3, 0, H, opts=cg.opts(loss=loss), ws=ws)
    cg.casgd_check(ws)
    assert torch.equal(x1, xl[:, 0])


@pytest.mark.parametrize("loss", ["logistic", "linear", "poisson"])
def test_csr_equals_dense_on_densified_matrix(cg, sparse, loss):
    p = sparse["linear" if loss == "logistic" else loss]
    m = 800
    rp = p.row_ptr[:m + 1]
    ci, va = p.col_idx[:rp[-1]], p.values[:rp[-1]]
    cols = np.unique(ci)[:200]
    keep = np.isin(ci, cols)
    remap = -np.ones(p.n, np.int64)
    remap[cols] = np.arange(cols.size)
    rows = np.repeat(np.arange(m), np.diff(rp))[keep]
    n = cols.size
    D = np.zeros((m, n), np.float32)
    D[rows, remap[ci[keep]]] = va[keep]
    y = p.y[:m] if loss != "logistic" else np.where(p.y[:m] >= 0, 1.0, -1.0).astype(np.float32)
    # CSR of the densified matrix
    nz = D != 0
    crp = np.concatenate([[0], np.cumsum(nz.sum(1))]).astype(np.int64)
    cci = np.nonzero(nz)[1].astype(np.int32)
    cva = D[nz].astype(np.float32)
    b, s, H, eta = 8, 4, 30, ETA_CSR[loss] / 4
    Xc = cg.csr_matrix(_dev(crp), _dev(cci), _dev(cva), n)
    ws = cg.casgd_sparse_prepare(Xc, b, s)
    xc = torch.zeros(n, device="cuda")
    cg.casgd_fit(Xc, _dev(y), xc, eta, 1e-3, b, s, 4, 0, H, opts=cg.opts(loss=loss), ws=ws)
    cg.casgd_check(ws)
    xd = torch.zeros(n, device="cuda")
    Xd = cg.dense_matrix(_dev(np.ascontiguousarray(D)))
    wsd = cg.casgd_fit(Xd, _dev(y), xd, eta, 1e-3, b, s, 4, 0, H, opts=cg.opts(loss=loss))
    cg.casgd_check(wsd)
    xo = R.casgd(D.astype(np.float64), y.astype(np.float64), np.zeros(n), eta, 1e-3, b, s, 4, 0,
                 H, loss=loss)
    for xv in (xc, xd):
        g = xv.cpu().numpy().astype(np.float64)
        assert np.linalg.norm(g - xo) / np.linalg.norm(xo) < 1e-4


@pytest.mark.parametrize("loss", ["linear", "poisson"])
def test_batched_launch_equals_solo_fits(cg, loss):
    """Problems with the linear or Poisson loss in one batched launch equal
    their solo fits bitwise (same variant), and the oracle to rounding."""
    probs = []
    for i, (m, n) in enumerate([(3000, 136), (5000, 72), (2000, 256)]):
        p = dense_glm(m, n, 40 + i, loss, var=1 / n, dtype=np.float32)
        probs.append(p)
    b, s, H, eta = 32, 4, 12, {"linear": 0.1, "poisson": 0.05}[loss]
    batch, xs = [], []
    for i, p in enumerate(probs):
        x = torch.zeros(p.X.shape[1], device="cuda")
        xs.append(x)
        batch.append(dict(X=cg.dense_matrix(_dev(p.X)), y=_dev(p.y), x=x, eta=eta, lam=1e-4, b=b,
                          s=s, seed=7 + i, n_outer=H, variant=2, loss=loss))
    wss = cg.casgd_fit_batch(batch)
    for w in wss:
        cg.casgd_check(w)
    for i, p in enumerate(probs):
        solo = torch.zeros(p.X.shape[1], device="cuda")
        w = cg.casgd_fit(cg.dense_matrix(_dev(p.X)), _dev(p.y), solo, eta, 1e-4, b, s, 7 + i, 0, H,
                         opts=cg.opts(exec_mode=1, fused_variant=2, loss=loss))
        cg.casgd_check(w)
        assert torch.equal(solo, xs[i])
        xo = R.casgd(p.X, p.y, np.zeros(p.X.shape[1]), eta, 1e-4, b, s, 7 + i, 0, H, loss=loss)
        g = xs[i].cpu().numpy().astype(np.float64)
        assert np.linalg.norm(g - xo) / np.linalg.norm(xo) < 1e-4


@pytest.mark.parametrize("loss", ["logistic", "linear", "poisson"])
@pytest.mark.parametrize("fmt", ["f32", "bf16"])
def test_loss_evaluation_vs_oracle(cg, loss, fmt):
    p = dense_glm(3000, 200, 8, loss, var=1 / 200, dtype=np.float32)
    codes = {"f32": cg.F32, "bf16": cg.BF16}[fmt]
    v, sc = cg.casgd_quantize(_dev(p.X), codes)
    X = cg.dense_matrix(v, sc, n=200)
    exact = R.quantize(p.X, fmt)[2]
    xs = (np.random.default_rng(2).standard_normal((3, 200)) * 0.3).astype(np.float32)
    got = cg.casgd_loss(X, _dev(p.y), _dev(xs), loss=loss).cpu().numpy()
    for k in range(3):
        ref = R.loss_value(exact, p.y.astype(np.float64), xs[k].astype(np.float64), loss)
        # margins accumulated in FP32 (gamma_n), terms and sum in FP64
        assert abs(got[k] - ref) <= 1e-5 * max(1.0, abs(ref)), (k, got[k], ref)
    if loss == "logistic":
        ll = cg.casgd_logloss(X, _dev(p.y), _dev(xs)).cpu().numpy()
        assert np.array_equal(ll, got)


@pytest.mark.parametrize("loss", ["linear", "poisson"])
def test_csr_loss_evaluation_vs_oracle(cg, sparse, loss):
    p = sparse[loss]
    X = cg.csr_matrix(_dev(p.row_ptr), _dev(p.col_idx), _dev(p.values), p.n)
    x = (np.random.default_rng(5).standard_normal(p.n) * 0.2).astype(np.float32)
    got = float(cg.casgd_loss(X, _dev(p.y), _dev(x), loss=loss))
    ref = R.loss_value_csr(p.row_ptr, p.col_idx, p.values, p.y, x.astype(np.float64), loss)
    assert abs(got - ref) <= 1e-5 * max(1.0, abs(ref))
