"""Many uneven problems in one fused launch (MI355X): every problem equals its
own solo fit bit for bit, and the solo fits match the FP64 oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import reference as R  # noqa: E402
from workloads import uneven_problem, uneven_problem_specs  # noqa: E402


@pytest.fixture(scope="module")
def cg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_18463_amd as cg
    cg._lib.load()
    return cg


def _problems(cg, count, seed, fmt, scale_m=0.1):
    specs = uneven_problem_specs(count, seed, m_range=(1e4 * scale_m, 2e5 * scale_m),
                                 n_range=(64, 1024))
    out = []
    code = {"f32": cg.F32, "bf16": cg.BF16, "fp8": cg.FP8E4M3}[fmt]
    for i, sp in enumerate(specs):
        p = uneven_problem(sp)
        src = torch.from_numpy(p.X).cuda()
        stored, scale = cg.casgd_quantize(src, code)
        X = cg.dense_matrix(stored, scale, n=p.n)
        _, _, exact = R.quantize(p.X, fmt)
        b, s = [(16, 4), (32, 8), (8, 1), (64, 16)][i % 4]
        # Step size scaled to the mean squared row norm (column scales reach
        # 10^3): a larger step makes the iteration amplify rounding
        # differences exponentially, and no two precisions stay comparable.
        eta = 0.5 / float((exact ** 2).sum(axis=1).mean())
        out.append(dict(p=p, X=X, exact=exact, y=torch.from_numpy(p.y).cuda(), b=b, s=s,
                        eta=eta, lam=1e-5, seed=100 + i, H=max(3, 400 // s)))
    return out


@pytest.mark.parametrize("fmt", ["f32", "bf16"])
def test_batch_equals_solo_and_oracle(cg, fmt):
    probs = _problems(cg, 7, 5, fmt)
    xs = [torch.zeros(q["p"].n, device="cuda") for q in probs]
    batch = [dict(X=q["X"], y=q["y"], x=xs[i], eta=q["eta"], lam=q["lam"], b=q["b"], s=q["s"],
                  seed=q["seed"], n_outer=q["H"], variant=2 if q["s"] > 1 else 1, gram_tile=64)
             for i, q in enumerate(probs)]
    wss = cg.casgd_fit_batch(batch)
    for ws in wss:
        cg.casgd_check(ws)
    for i, q in enumerate(probs):
        solo = torch.zeros(q["p"].n, device="cuda")
        o = cg.opts(exec_mode=1, fused_variant=batch[i]["variant"], gram_tile=64)
        cg.casgd_fit(q["X"], q["y"], solo, q["eta"], q["lam"], q["b"], q["s"], q["seed"], 0,
                     q["H"], opts=o)
        assert torch.equal(solo, xs[i]), i
        xo = R.casgd(q["exact"], q["p"].y, np.zeros(q["p"].n), q["eta"], q["lam"], q["b"],
                     q["s"], q["seed"], 0, q["H"])
        xg = xs[i].cpu().numpy().astype(np.float64)
        assert np.linalg.norm(xg - xo) / max(np.linalg.norm(xo), 1e-30) < 1e-4, i


def test_batch_explicit_groups(cg):
    probs = _problems(cg, 3, 9, "f32")
    xs = [torch.zeros(q["p"].n, device="cuda") for q in probs]
    batch = [dict(X=q["X"], y=q["y"], x=xs[i], eta=q["eta"], lam=q["lam"], b=q["b"], s=q["s"],
                  seed=q["seed"], n_outer=q["H"], groups=3, variant=2 if q["s"] > 1 else 1,
                  gram_tile=64)
             for i, q in enumerate(probs)]
    for ws in cg.casgd_fit_batch(batch):
        cg.casgd_check(ws)
    for i, q in enumerate(probs):
        solo = torch.zeros(q["p"].n, device="cuda")
        o = cg.opts(exec_mode=1, fused_variant=batch[i]["variant"], gram_tile=64)
        cg.casgd_fit(q["X"], q["y"], solo, q["eta"], q["lam"], q["b"], q["s"], q["seed"], 0,
                     q["H"], opts=o)
        assert torch.equal(solo, xs[i]), i


def test_full_size_uneven_batch_sampled_check(cg):
    """The full uneven workload shape: 64 problems, m log-uniform in
    [10^4, 2*10^5], n in [128, 4096], column-scale spread up to 10^3, BF16
    storage, b = 64, s = 16, all in one batched launch (automatic groups and
    forms). Three outer iterations; four problems (the smallest and largest
    m and n) checked against the oracle on the stored values of their sampled
    rows, which is all the oracle reads."""
    b, s, H, lam = 64, 16, 3, 1e-5
    specs = uneven_problem_specs(64, 2024)
    pick = {int(np.argmin([q["m"] for q in specs])), int(np.argmax([q["m"] for q in specs])),
            int(np.argmin([q["n"] for q in specs])), int(np.argmax([q["n"] for q in specs]))}
    batch, keep = [], {}
    for i, sp in enumerate(specs):
        p = uneven_problem(sp)
        stored, scale = cg.casgd_quantize(torch.from_numpy(p.X).cuda(), cg.BF16)
        X = cg.dense_matrix(stored, scale, n=p.n)
        # step size from the mean squared row norm of a row sample (as the
        # driver of the learned preconditioner does for its plain baseline)
        rows = p.X[:: max(1, p.m // 2048)].astype(np.float64)
        eta = 0.5 / float((rows ** 2).sum(axis=1).mean())
        x = torch.zeros(p.n, device="cuda")
        batch.append(dict(X=X, y=torch.from_numpy(p.y).cuda(), x=x, eta=eta, lam=lam, b=b, s=s,
                          seed=300 + i, n_outer=H))
        if i in pick:
            idx = np.unique(R.sample_indices(300 + i, 0, H * s * b, p.m))
            _, _, exact = R.quantize(p.X[idx], "bf16")
            p.X[idx] = exact
            keep[i] = (p, eta)
        del p
    for ws in cg.casgd_fit_batch(batch):
        cg.casgd_check(ws)
    for i, (p, eta) in keep.items():
        xo = R.casgd(p.X, p.y, np.zeros(p.n), eta, lam, b, s, 300 + i, 0, H)
        xg = batch[i]["x"].cpu().numpy().astype(np.float64)
        err = np.linalg.norm(xg - xo) / max(np.linalg.norm(xo), 1e-30)
        print(f"\n[c5 scale] problem {i} m={p.m} n={p.n} rel_err={err:.3e}")
        assert err < 1e-4, i


@pytest.mark.parametrize("fmt", ["f32", "bf16"])
@pytest.mark.parametrize("gram_tile", [64, 128])
def test_batch_variant3_equals_solo(cg, fmt, gram_tile):
    """The chain + helper recurrence (fused variant 3) inside each problem's
    workgroup group: automatic form and explicit groups, bitwise equal to
    the solo fused variant 3 fits (the result does not depend on how many
    workgroups share the Gram and update work), with snapshots per problem."""
    probs = [q for q in _problems(cg, 8, 13, fmt) if q["s"] >= 4]
    xs = [torch.zeros(q["p"].n, device="cuda") for q in probs]
    hists = [torch.zeros(q["H"], q["p"].n, device="cuda") for q in probs]
    ths = [torch.zeros(q["H"] + 1, dtype=torch.int64, device="cuda") for q in probs]
    batch = [dict(X=q["X"], y=q["y"], x=xs[i], eta=q["eta"], lam=q["lam"], b=q["b"], s=q["s"],
                  seed=q["seed"], n_outer=q["H"], snapshot_every=1, x_history=hists[i],
                  t_history=ths[i], groups=(0 if i % 2 else 20), gram_tile=gram_tile)
             for i, q in enumerate(probs)]
    for ws in cg.casgd_fit_batch(batch):
        cg.casgd_check(ws)
    for i, q in enumerate(probs):
        solo = torch.zeros(q["p"].n, device="cuda")
        o = cg.opts(exec_mode=1, fused_variant=3, gram_tile=gram_tile)
        cg.casgd_fit(q["X"], q["y"], solo, q["eta"], q["lam"], q["b"], q["s"], q["seed"], 0,
                     q["H"], opts=o)
        assert torch.equal(solo, xs[i]), i
        assert torch.equal(hists[i][-1], xs[i])
        t = ths[i].cpu().numpy()
        assert np.all(np.diff(t) >= 0) and t[-1] > t[0]
