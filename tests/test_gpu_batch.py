"""Batched persistent CG (needs an MI355X).

Many independent unit-cube problems solved in one persistent launch are
compared with the oracle's direct solves (problems small enough for the
dense oracle, every degree 1..10, every tile variant), with single-problem
GPU solves, and, at the full 256-problem size, through oracle residuals on
the smallest problems and single-problem solves on a sample.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from helpers import gpu_ctx, rel_err, to_dev, to_host

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def _small_problems():
    """Every degree 1..10 on meshes of 1..3 elements per axis (one problem
    without interior faces), lambda log-uniform in [1e-2, 1e2], f ~ N(0,1)."""
    rng = np.random.default_rng(41)
    out = []
    for p in list(range(1, 11)) + [3, 2]:
        n = tuple(int(v) for v in rng.integers(1, 4, size=3))
        if p == 10:
            n = (2, 2, 1)
        out.append((n, p, float(10.0 ** rng.uniform(-2, 2))))
    out.append(((1, 1, 1), 4, 0.5))
    return out


def _batch_inputs(specs, seed):
    import paper_2007_11891_amd as pkg
    b = pkg.HdgBatch([s[0] for s in specs], [s[1] for s in specs], [s[2] for s in specs], tau=1.0)
    f = np.random.default_rng(seed).standard_normal(b.total_vol)
    return b, f


@pytest.fixture(scope="module")
def small():
    specs = _small_problems()
    b, f = _batch_inputs(specs, 17)
    refs = []
    for i, (n, p, lam) in enumerate(specs):
        print(f"[batch oracle] problem {i} n={n} p={p} lam={lam:.3g}", flush=True)
        widths = [W.uniform_widths(v) for v in n]
        o = oracle.HdgOracle(n, widths, p, 1.0, np.full(n[0] * n[1] * n[2], lam))
        fi = f[b.vol_off[i]:b.vol_off[i + 1]]
        ut = o.solve(fi, np.zeros(o.layout.n_all))
        refs.append((ut[:o.layout.n_free], o.reconstruct(fi, ut)))
    return specs, b, f, refs


@pytest.mark.parametrize("form", [0, 1, 2])
@pytest.mark.parametrize("variant", [0, 1, 2])
def test_batch_matches_oracle_every_degree_and_tile(small, variant, form):
    import paper_2007_11891_amd as pkg
    specs, b, f, refs = small
    print(f"[batch vs oracle] tile variant {variant} form {form}", flush=True)
    b.set_form(form)
    assert b.form() == form
    b.set_tile(0, variant)
    assert set(b.tiles().values()) == {variant}
    opts = pkg.default_opts(rtol=1e-15, maxit=1500)
    tr, uv, res, ms = b.solve_forcing(to_dev(f), opts=opts, allow_noconv=True)
    tr, uv = to_host(tr), to_host(uv)
    for i, (ut_ref, uv_ref) in enumerate(refs):
        assert res[i]["status"] in (0, -4), (i, res[i])
        t = tr[b.free_off[i]:b.free_off[i + 1]]
        u = uv[b.vol_off[i]:b.vol_off[i + 1]]
        if ut_ref.size:
            assert rel_err(t, ut_ref) < 1e-12, (i, specs[i], res[i])
        assert rel_err(u, uv_ref) < 1e-12, (i, specs[i], res[i])
    b.set_tile(0, 0)
    b.set_form(0)


@pytest.mark.parametrize("form", [0, 1, 2])
def test_problem_without_interior_faces_converges_at_once(small, form):
    import paper_2007_11891_amd as pkg
    specs, b, f, refs = small
    b.set_form(form)
    _, _, res, _ = b.solve_forcing(to_dev(f), opts=pkg.default_opts(rtol=1e-10))
    b.set_form(0)
    i = len(specs) - 1
    assert b.n_free[i] == 0
    assert res[i]["status"] == 0 and res[i]["iters"] == 0


@pytest.mark.parametrize("form", [0, 1, 2])
def test_batch_matches_single_problem_solves_and_is_deterministic(small, form):
    import paper_2007_11891_amd as pkg
    specs, b, f, _ = small
    print(f"[batch vs single] form {form}", flush=True)
    b.set_form(form)
    opts = pkg.default_opts(rtol=1e-10, maxit=5000)
    tr1, uv1, res1, _ = b.solve_forcing(to_dev(f), opts=opts)
    tr2, uv2, res2, _ = b.solve_forcing(to_dev(f), opts=opts)
    assert torch.equal(tr1, tr2) and torch.equal(uv1, uv2)
    assert [r["iters"] for r in res1] == [r["iters"] for r in res2]
    for i, (n, p, lam) in enumerate(specs):
        c = gpu_ctx(n, [W.uniform_widths(v) for v in n], p, 1.0, lam)
        fi = to_dev(f[b.vol_off[i]:b.vol_off[i + 1]])
        t, u, info = c.solve_forcing(fi, c.zeros_trace(), opts=opts)
        nf = c.sizes.n_free
        assert abs(info["iters"] - res1[i]["iters"]) <= 2, (i, info, res1[i])
        if nf:
            assert rel_err(to_host(tr1[b.free_off[i]:b.free_off[i + 1]]), to_host(t)[:nf]) < 1e-8
        assert rel_err(to_host(uv1[b.vol_off[i]:b.vol_off[i + 1]]), to_host(u)) < 1e-8
        assert res1[i]["rel_res"] <= 1e-10
    b.set_form(0)


def test_batch_iteration_cap_reported_in_every_form(small):
    """maxit = 3: a problem that needs more stops with ENOCONV after exactly
    3 iterations, in every form (tiny ones may converge within 3)."""
    import paper_2007_11891_amd as pkg
    specs, b, f, _ = small
    for form in (0, 1, 2):
        b.set_form(form)
        _, _, res, _ = b.solve_forcing(to_dev(f), opts=pkg.default_opts(rtol=1e-14, maxit=3),
                                       allow_noconv=True)
        for i, r in enumerate(res):
            if b.n_free[i]:
                assert (r["status"] == -4 and r["iters"] == 3) or \
                       (r["status"] == 0 and r["iters"] <= 3), (form, i, r)
        assert sum(r["status"] == -4 for r in res) >= len(res) // 2
    b.set_form(0)


def test_batch_rejects_mixed_precision(small):
    import paper_2007_11891_amd as pkg
    specs, b, f, _ = small
    with pytest.raises(pkg.HdgError, match="EUNSUPPORTED"):
        b.solve_forcing(to_dev(f), opts=pkg.default_opts(mixed=1))


# ------------------------------- full size -----------------------------------
@pytest.fixture(scope="module")
def full():
    import paper_2007_11891_amd as pkg
    probs = W.batched()
    b = pkg.HdgBatch([pr.n for pr in probs], [pr.p for pr in probs],
                     [float(pr.lam[0]) for pr in probs], tau=1.0)
    f = np.concatenate([pr.f_values for pr in probs])
    return probs, b, f


def test_full_batch_converges_and_matches_samples(full):
    """256 problems (sizes 4..12 per axis, p 2..10) in the launch the bench
    times, autotuned tiles: every problem converges to 1e-10; sampled
    problems equal their single-problem solves; the smallest ones have
    small oracle residuals."""
    import paper_2007_11891_amd as pkg
    probs, b, f = full
    print(f"[batch full] {len(probs)} problems, {b.total_free} free DOFs", flush=True)
    tiles = b.autotune(iters=10, reps=2)
    print(f"[batch full] tiles {tiles}", flush=True)
    opts = pkg.default_opts(rtol=1e-10, maxit=20000)
    tr, uv, res, ms = b.solve_forcing(to_dev(f), opts=opts)
    print(f"[batch full] {ms:.2f} ms, max iters {max(r['iters'] for r in res)}", flush=True)
    assert all(r["status"] == 0 and r["rel_res"] <= 1e-10 for r in res)
    rng = np.random.default_rng(3)
    for i in sorted(rng.choice(len(probs), size=6, replace=False)):
        pr = probs[i]
        print(f"[batch full] single-problem check {i} n={pr.n} p={pr.p}", flush=True)
        c = gpu_ctx(pr.n, pr.widths, pr.p, 1.0, float(pr.lam[0]))
        t, u, info = c.solve_forcing(to_dev(pr.f_values), c.zeros_trace(), opts=opts)
        nf = c.sizes.n_free
        assert abs(info["iters"] - res[i]["iters"]) <= 2, (i, info, res[i])
        assert rel_err(to_host(tr[b.free_off[i]:b.free_off[i + 1]]), to_host(t)[:nf]) < 1e-8
        assert rel_err(to_host(uv[b.vol_off[i]:b.vol_off[i + 1]]), to_host(u)) < 1e-8
    # oracle residual of the nodal trace on the two cheapest problems
    cost = [pr.n[0] * pr.n[1] * pr.n[2] * (pr.p + 1) ** 3 for pr in probs]
    for i in np.argsort(cost)[:2]:
        pr = probs[i]
        print(f"[batch full] oracle residual {i} n={pr.n} p={pr.p}", flush=True)
        o = oracle.HdgOracle(pr.n, pr.widths, pr.p, 1.0, pr.lam)
        nf = o.layout.n_free
        F = o.lifted_rhs(pr.f_values, np.zeros(o.layout.n_all))
        x = np.zeros(o.layout.n_all)
        x[:nf] = to_host(tr[b.free_off[i]:b.free_off[i + 1]])
        K = o.assemble_K()
        r = F - K[:nf, :nf] @ x[:nf]
        assert np.linalg.norm(r) / np.linalg.norm(F) < 1e-9
