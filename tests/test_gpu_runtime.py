"""GPU: the runtime around the kernels -- launch shapes, table batching,
timing mode and its work counts, the launch-shape autotuner -- each checked
against the CPU oracle (same bar as the parity tests)."""
import os

import numpy as np
import pytest

import oracle
import workloads as w

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2608_01467_amd as fhs  # noqa: E402
from paper_2608_01467_amd import tune  # noqa: E402

TOL = 1e-12
THREADS = min(16, len(os.sched_getaffinity(0)))


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = fhs.Context(0)
    yield c
    c.set_launch_config(0, 0, 0)


def _cases():
    walk = w.quantum_walk(99, 7).to_text()
    qaoa = w.qaoa_maxcut(8, 2, 11, 12)[0].to_text()
    return [("walk", walk, w.walk_outputs(99, 7, 40, seed=5), 0.0),
            ("qaoa", qaoa, list(range(0, 256, 3)), 1e-4)]


def _run(ctx, prog, outs, thr, part):
    ctx.load(prog)
    ctx.set_partition(*part)
    amps, st = ctx.evaluate([0], [1], outs, threshold=thr)
    torch.cuda.synchronize()
    a = amps.cpu().numpy()
    return a[:, 0] + 1j * a[:, 1], st.cpu().numpy().view(np.uint64)


def _check(name, amps, st, ref):
    assert np.abs(amps - ref[0]).max() <= TOL, name
    assert np.array_equal(st[:, :3], ref[1][:, :3].astype(np.uint64)), name


@pytest.mark.parametrize("case", [0, 1])
def test_launch_shapes(ctx, case):
    """Every histories-per-lane x chunk x blocks-per-CU shape gives the
    oracle's amplitudes and bit-identical valid-set statistics."""
    name, text, outs, thr = _cases()[case]
    prog = fhs.Program(text)
    part = prog.choose_partition(fhs.PART_EQ8)
    ref = oracle.Feynman(text).evaluate([0], [1], outs, threshold=thr, threads=THREADS)
    for h in (1, 2):
        for chunk in (1, 64, 256):
            for bpc in (0, 1, 3):
                for dispatch in ((0, 1, 2, 3) if chunk == 64 else (0,)):
                    ctx.set_launch_config(h, chunk, bpc, dispatch)
                    assert ctx.launch_config == (h, chunk, bpc, dispatch)
                    amps, st = _run(ctx, prog, outs, thr, part)
                    _check((name, h, chunk, bpc, dispatch), amps, st, ref)
    # the plain form under both dispatch granularities
    for dispatch in (1, 2):
        ctx.set_launch_config(2, 0, 0, dispatch)
        ctx.load(prog)
        amps, st = ctx.evaluate([0], [1], outs, threshold=thr, plain=True)
        torch.cuda.synchronize()
        a = amps.cpu().numpy()
        _check((name, "plain", dispatch), a[:, 0] + 1j * a[:, 1],
               st.cpu().numpy().view(np.uint64), ref)
    ctx.set_launch_config(0, 0, 0)
    with pytest.raises(fhs.FhsError):
        ctx.set_launch_config(3, 0, 0)
    with pytest.raises(fhs.FhsError):
        ctx.set_launch_config(1, 96, 0)       # not a power of two
    with pytest.raises(fhs.FhsError):
        ctx.set_launch_config(1, 64, 0, 4)    # no such dispatch mode


def test_table_batches_and_timing(ctx):
    """A table budget of a few pairs splits the work into many batches (one
    prefix build + consumer launch each); results are unchanged, timing
    mode reports one duration per batch, and the work counts are exact."""
    text = w.quantum_walk(99, 14).to_text()        # A = 13: 2^13 entries per pair
    outs = w.walk_outputs(99, 14, 12, seed=5)
    prog = fhs.Program(text)
    ref = oracle.Feynman(text).evaluate([0], [1], outs, threads=THREADS,
                                        partition=prog.choose_partition(fhs.PART_EQ8))
    ctx.load(prog)
    for part in ((prog.G, prog.G), prog.choose_partition(fhs.PART_EQ8)):
        ctx.set_partition(*part)
        plan1 = ctx.plan(len(outs), 1)
        assert plan1["n_batches"] == 1
        assert plan1["Ap"] + plan1["Ar"] + plan1["As"] == prog.A
        per_pair = plan1["table_bytes"] // plan1["pairs_per_batch"]
        budget = max(1 << 20, 3 * per_pair)
        ctx.set_table_budget(budget)
        plan = ctx.plan(len(outs), 1)
        B = min(len(outs), budget // per_pair)
        assert plan["pairs_per_batch"] == B
        assert plan["n_batches"] == (len(outs) + B - 1) // B
        amps, st = _run(ctx, prog, outs, 0.0, part)
        _check(("batched", part), amps, st, ref)
        ctx.set_kernel_timing(True)
        amps, st = _run(ctx, prog, outs, 0.0, part)
        _check(("timed", part), amps, st, ref)
        times = ctx.kernel_times()
        assert len(times) == plan["n_batches"] and all(t > 0 for t in times)
        entries, valid = ctx.kernel_counts()
        assert entries == len(outs) << plan["Ap"]
        assert 0 < valid <= entries
        if part == (prog.G, prog.G):
            # all sources in the prefix: a consistent entry is a valid history
            assert plan["Ap"] == prog.A
            assert valid == int(ref[1][:, 0].sum())
        ctx.set_kernel_timing(False)
        ctx.set_table_budget(1 << 30)


@pytest.mark.parametrize("case", [0, 1])
def test_items_per_claim(ctx, case):
    """A consumer workgroup may take several work items per atomic on the
    queue's counter: every claim size (and the automatic one) gives the
    oracle's amplitudes and valid sets, including claims that run past the
    last item; the plan reports the size in use."""
    name, text, outs, thr = _cases()[case]
    prog = fhs.Program(text)
    part = prog.choose_partition(fhs.PART_EQ8)
    ref = oracle.Feynman(text).evaluate([0], [1], outs, threshold=thr, threads=THREADS)
    for dispatch in (0, 3):
        for claim in (0, 1, 3, 16, 64):
            ctx.set_launch_config(2, 4, 0, dispatch, claim)
            assert ctx.items_per_claim == claim
            amps, st = _run(ctx, prog, outs, thr, part)
            plan = ctx.plan(len(outs), 1)
            assert plan["items_per_claim"] == (claim or plan["items_per_claim"]) >= 1
            _check((name, dispatch, claim), amps, st, ref)
    ctx.set_launch_config(0, 0, 0, 0)


def test_autotune_launch(ctx):
    name, text, outs, thr = _cases()[1]
    wl = tune.Workload(ctx, text, [0], [1.0], outs, thr)
    part = wl.prog.choose_partition(fhs.PART_EQ8)
    best, log = tune.autotune_launch(wl, part, reps=1)
    # 18 automatic-dispatch shapes, 3 dispatch modes, then the compiled
    # consumer's histories-per-lane x chunk (one may repeat an earlier entry)
    cfgs = [c for c, _ in log]
    assert len(log) in (24, 25) and len(set(cfgs)) == len(cfgs) and best in cfgs
    assert ctx.launch_config == best
    ref = oracle.Feynman(text).evaluate([0], [1], outs, threshold=thr, threads=THREADS)
    wl.run(part)
    torch.cuda.synchronize()
    a = wl.amps.cpu().numpy()
    _check("autotuned", a[:, 0] + 1j * a[:, 1], wl.stats.cpu().numpy().view(np.uint64), ref)
    ctx.set_launch_config(0, 0, 0)


def test_literal_aa16_split_choice(ctx):
    """Amplitude amplification with 16 + 14 qubits (A = 96): only the split
    choice runs -- features, Eq. (8), the model's predictions (outside its
    training range: NaN, and FHS_ERANGE for the model's choice)."""
    text = w.amplitude_amplification(16, 3, 4, 301)[0].to_text()
    prog = fhs.Program(text)
    assert prog.A == 96
    cand = prog.candidate_splits()
    assert len(cand) == 97 * 98 // 2
    f = prog.split_features(*prog.choose_partition(fhs.PART_EQ8), 64, 1)
    assert np.isfinite(f).all() and f[12] > 64     # Eq. (8) cost beyond 2^64, in 128 bits
    ctx.load(prog)
    blob = tune.load_model()
    if blob is None:
        pytest.skip("no trained cost model in the package")
    ctx.load_cost_model(blob)
    assert np.isnan(ctx.predict_splits(cand[:50], 64, 1)).all()
    with pytest.raises(fhs.FhsError) as e:
        ctx.choose_partition(fhs.PART_MODEL, 64, 1)
    assert e.value.status == 3


def test_precompile(ctx):
    """fhs_precompile builds the compiled consumers of many splits on host
    threads; the evaluations then use them (and still match the oracle)."""
    name, text, outs, thr = _cases()[1]
    prog = fhs.Program(text)
    ctx.load(prog)
    cand = prog.candidate_splits()[:12]
    ctx.set_launch_config(1, 0, 0, 0)
    assert ctx.precompile(cand, len(outs), 1, thr) == 0          # not compiled mode: nothing to do
    ctx.set_launch_config(1, 0, 0, 3)
    n = ctx.precompile(cand, len(outs), 1, thr, threads=8)
    assert 1 <= n <= len(cand)
    assert ctx.precompile(cand, len(outs), 1, thr) == 0          # all cached now
    ref = oracle.Feynman(text).evaluate([0], [1], outs, threshold=thr, threads=THREADS)
    for c in cand[:4]:
        ctx.set_partition(*c)
        amps, st = ctx.evaluate([0], [1], outs, threshold=thr)
        torch.cuda.synchronize()
        a = amps.cpu().numpy()
        assert np.abs(a[:, 0] + 1j * a[:, 1] - ref[0]).max() <= 1e-12, c
        assert np.array_equal(st.cpu().numpy().view(np.uint64)[:, :3], ref[1][:, :3].astype(np.uint64))
    with pytest.raises(fhs.FhsError):
        ctx.precompile([(5, 2)], len(outs), 1, thr)
    ctx.set_launch_config(0, 0, 0, 0)


def test_workspace_too_small(ctx):
    """fhs_evaluate and fhs_evaluate_plain with a workspace below
    fhs_workspace_size: FHS_ENOMEM (status 4), nothing launched, the outputs
    left as they were; with the full size the same call succeeds."""
    import ctypes
    name, text, outs, thr = _cases()[0]
    prog = fhs.Program(text)
    ctx.load(prog)
    ctx.set_partition(*prog.choose_partition(fhs.PART_EQ8))
    d_in, d_out = ctx.device_bits([0]), ctx.device_bits(outs)
    d_cf = ctx.device_coeffs([1.0])
    M = len(outs)
    need = ctx.workspace_size(M, 1)
    assert need > 256
    ws = torch.empty(need, dtype=torch.uint8, device="cuda:0")
    amps = torch.full((M, 2), 7.0, dtype=torch.float64, device="cuda:0")
    stats = torch.full((M, 4), 7, dtype=torch.int64, device="cuda:0")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    L = fhs.lib()
    for fn in (L.fhs_evaluate, L.fhs_evaluate_plain):
        st = fn(ctx._h, d_in.data_ptr(), d_cf.data_ptr(), 1, d_out.data_ptr(), M, float(thr),
                amps.data_ptr(), stats.data_ptr(), ws.data_ptr(), need - 256, stream)
        assert st == 4, st
        assert b"workspace" in L.fhs_last_error(ctx._h)
        torch.cuda.synchronize()
        assert bool((amps == 7.0).all()) and bool((stats == 7).all())
    st = L.fhs_evaluate(ctx._h, d_in.data_ptr(), d_cf.data_ptr(), 1, d_out.data_ptr(), M, float(thr),
                        amps.data_ptr(), stats.data_ptr(), ws.data_ptr(), need, stream)
    assert st == 0
    torch.cuda.synchronize()
    ref = oracle.Feynman(text).evaluate([0], [1], outs, threshold=thr, threads=THREADS)
    a = amps.cpu().numpy()
    _check("full workspace", a[:, 0] + 1j * a[:, 1], stats.cpu().numpy().view(np.uint64), ref)
