"""The autotuner: a solve tunes its shape once (every candidate timed on the
problem's own codes, the choice kept and reported), and every pass candidate
computes the same iterates bit for bit (they change the launch shape, not the
arithmetic of any column)."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1802_04907_amd as qiht  # noqa: E402
import workloads  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
# instance (cache: two waves per SIMD, long: three) x spans per workgroup in the
# pass's span queue (r2 and up: workgroups take further spans from the queue)
PASS_CANDIDATES = [f"{inst}/r{r}" for inst in ("cache", "long") for r in (1, 2, 4, 8)]


def _gpu(p, bits):
    q = qiht.quantize_matrix(torch.from_numpy(p.phi).to(DEV), bits, 2, p.seed)
    yhat, _, _ = qiht.quantize_vector(torch.from_numpy(p.y).to(DEV), 32 if bits == 32 else 8, p.seed)
    return q, yhat


@pytest.mark.parametrize("bits", [2, 4, 8, 32])
def test_pass_candidates_give_identical_solves(monkeypatch, bits):
    p = workloads.gaussian(2000, 7000, 70, 1e-3, seed=41 + bits, dtype=np.float32)
    q, yhat = _gpu(p, bits)
    x0, s0, i0 = qiht.niht_solve(q, yhat, p.s, max_iters=40, tol=-1.0)  # tunes this shape
    rep = qiht.tune_report()["entries"]
    mine = [e for e in rep if f"|pass|bits{bits}|count1|" in e["key"] and f"|n{q.n}|" in e["key"]]
    assert len(mine) == 1, rep
    e = mine[0]
    assert set(e["candidates_us"]) == set(PASS_CANDIDATES)
    assert all(v > 0 for v in e["candidates_us"].values())
    assert e["choice"] in PASS_CANDIDATES and e["default"] in PASS_CANDIDATES
    for cand in PASS_CANDIDATES:
        monkeypatch.setenv("QIHT_TUNE_FORCE", cand)
        x, s, i = qiht.niht_solve(q, yhat, p.s, max_iters=40, tol=-1.0)
        assert torch.equal(x.view(torch.int32), x0.view(torch.int32)), cand
        assert torch.equal(s, s0), cand
        assert i["backtracks"] == i0["backtracks"] and i["mu_last"] == i0["mu_last"], cand
    q.free()


def test_batch_and_shared_gemm_are_tuned():
    ms = [600, 1100, 400]
    probs = [workloads.gaussian(m, 4 * m, m // 16, 1e-3, [9, i], np.float32, qseed=i)
             for i, m in enumerate(ms)]
    gpu = [(*_gpu(p, 4), p.s) for p in probs]
    qiht.niht_solve_batched(gpu, max_iters=5, tol=-1.0)
    rng = np.random.default_rng(3)
    phi = (rng.standard_normal((1024, 4096)) / 32.0).astype(np.float32)
    qd = qiht.quantize_matrix(torch.from_numpy(phi).to(DEV), qiht.BF16, 1, 0)
    ys = [torch.from_numpy(phi.astype(np.float64) @ rng.standard_normal(4096)).to(DEV) for _ in range(6)]
    qiht.niht_solve_batched([(qd, y, 16) for y in ys], max_iters=5, tol=-1.0)
    keys = [e["key"] for e in qiht.tune_report()["entries"]]
    assert any("|pass|bits4|count3|" in k for k in keys), keys
    gemm = [e for e in qiht.tune_report()["entries"] if "|gemm|" in e["key"] and "|count6|" in e["key"]]
    assert len(gemm) == 1 and gemm[0]["choice"].startswith("ks"), gemm
    for q, _, _ in gpu:
        q.free()
    qd.free()
