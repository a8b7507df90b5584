"""Rounds replayed as captured HIP graphs against the same rounds launched
one by one (QIHT_GRAPH=0): the kernels and their arguments are the same, so
x, the support and the solve's counters must be bitwise equal.  A launch
shape is captured once it recurs (from its third solve on), so each case runs
four solves with eager work and synchronizations in between: two launched
directly, then one that captures and replays, then one that replays the
cached executable graphs; every solve replays its chunk graphs many times
(16 rounds per chunk)."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1802_04907_amd as qiht  # noqa: E402
import workloads  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
FIELDS = ("iterations", "reason", "backtracks", "capped_iterations", "mu_last", "full_selects")


def _gpu(p, bits, ybits=8):
    q = qiht.quantize_matrix(torch.from_numpy(p.phi).to(DEV), bits, 2, p.seed)
    yhat, _, _ = qiht.quantize_vector(torch.from_numpy(p.y).to(DEV), ybits, p.seed)
    return q, yhat


def _same(a, b, label):
    xa, sa, ia = a
    xb, sb, ib = b
    assert torch.equal(xa.view(torch.int32), xb.view(torch.int32)), label
    assert torch.equal(sa, sb), label
    for f in FIELDS:
        assert ia[f] == ib[f], (label, f)


@pytest.mark.parametrize("bits", [4, 8, 32])
def test_single_solve_graph_equals_eager(monkeypatch, bits):
    p = workloads.gaussian(1500, 6000, 60, 1e-3, seed=31, dtype=np.float32)
    q, yhat = _gpu(p, bits, 32 if bits == 32 else 8)
    monkeypatch.setenv("QIHT_GRAPH", "0")
    ref = qiht.niht_solve(q, yhat, p.s, max_iters=100, tol=-1.0)
    monkeypatch.delenv("QIHT_GRAPH")
    for rep in range(4):
        got = qiht.niht_solve(q, yhat, p.s, max_iters=100, tol=-1.0)
        torch.cuda.synchronize()
        _same(ref, got, f"{bits}-bit replay {rep}")
        torch.zeros(1 << 20, device=DEV).add_(1.0)  # eager work between the solves
        torch.cuda.synchronize()
    q.free()


def test_batched_solve_graph_equals_eager(monkeypatch):
    ms = [700, 1200, 300, 900]
    probs = [workloads.gaussian(m, 4 * m, m // 16, 1e-3, [5, i], np.float32, qseed=i)
             for i, m in enumerate(ms)]
    gpu = [(*_gpu(p, 4), p.s) for p in probs]
    monkeypatch.setenv("QIHT_GRAPH", "0")
    ref = qiht.niht_solve_batched(gpu, max_iters=60, tol=-1.0)
    monkeypatch.delenv("QIHT_GRAPH")
    for rep in range(4):
        got = qiht.niht_solve_batched(gpu, max_iters=60, tol=-1.0)
        torch.cuda.synchronize()
        for i in range(len(ms)):
            _same(ref[i], got[i], f"batch problem {i} replay {rep}")
    for q, _, _ in gpu:
        q.free()


def test_pass_span_queue_in_graphs_equals_static_split(monkeypatch):
    """The full pass's span queue (8 spans per workgroup, forced) under graph
    replay: its counters are reset by each launch's last workgroup, so every
    replayed pass takes all its spans; the iterates equal the static split's
    (one span per workgroup, launched directly) bit for bit."""
    ms = [700, 1200, 300, 900]
    probs = [workloads.gaussian(m, 4 * m, m // 16, 1e-3, [6, i], np.float32, qseed=i)
             for i, m in enumerate(ms)]
    gpu = [(*_gpu(p, 4), p.s) for p in probs]
    monkeypatch.setenv("QIHT_GRAPH", "0")
    monkeypatch.setenv("QIHT_TUNE_FORCE", "long/r1")
    ref = qiht.niht_solve_batched(gpu, max_iters=60, tol=-1.0)
    monkeypatch.delenv("QIHT_GRAPH")
    monkeypatch.setenv("QIHT_TUNE_FORCE", "long/r8")
    for rep in range(4):
        got = qiht.niht_solve_batched(gpu, max_iters=60, tol=-1.0)
        torch.cuda.synchronize()
        for i in range(len(ms)):
            _same(ref[i], got[i], f"queue problem {i} replay {rep}")
        torch.zeros(1 << 20, device=DEV).add_(1.0)  # eager work between the solves
        torch.cuda.synchronize()
    for q, _, _ in gpu:
        q.free()


def test_shared_matrix_batch_graph_equals_eager(monkeypatch):
    rng = np.random.default_rng(7)
    m, n, s, nrhs = 600, 2400, 20, 8
    phi = (rng.standard_normal((m, n)) / np.sqrt(m)).astype(np.float32)
    q = qiht.quantize_matrix(torch.from_numpy(phi).to(DEV), qiht.BF16, 1, 0)
    ys = []
    for _ in range(nrhs):
        x = np.zeros(n)
        x[rng.choice(n, s, replace=False)] = rng.standard_normal(s)
        ys.append(torch.from_numpy(phi.astype(np.float64) @ x).to(DEV))
    probs = [(q, y, s) for y in ys]
    monkeypatch.setenv("QIHT_GRAPH", "0")
    ref = qiht.niht_solve_batched(probs, max_iters=40, tol=-1.0)
    monkeypatch.delenv("QIHT_GRAPH")
    for rep in range(4):
        got = qiht.niht_solve_batched(probs, max_iters=40, tol=-1.0)
        torch.cuda.synchronize()
        for i in range(nrhs):
            _same(ref[i], got[i], f"shared rhs {i} replay {rep}")
    q.free()


def test_profiled_solves_mix_timed_chunks_and_graphs():
    """profile = N times the first pass of every N-th chunk of 16 rounds
    (that round launched directly, the rest of the chunk replaying as a
    graph once the shape recurs): the results equal the unprofiled solve's
    bit for bit, and one launch is timed per timed chunk."""
    p = workloads.gaussian(1500, 6000, 60, 1e-3, seed=32, dtype=np.float32)
    q, yhat = _gpu(p, 4)
    ref = qiht.niht_solve(q, yhat, p.s, max_iters=100, tol=-1.0)
    for rep in range(4):
        x, sup, info = qiht.niht_solve(q, yhat, p.s, max_iters=100, tol=-1.0, profile=3)
        torch.cuda.synchronize()
        _same(ref, (x, sup, info), f"profiled solve {rep}")
        # 101 rounds = chunks of 16 x 6 + 5: chunks 0, 3 and 6 timed (more
        # chunks only if some iteration needed more than four shrinks)
        assert info["pass_launches"] >= 3, info
        avg_us = info["pass_ms"] * 1e3 / info["pass_launches"]
        assert 0.5 < avg_us < 5000.0, avg_us
    q.free()
