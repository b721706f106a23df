"""fhs_evaluate_noalloc (the entry point for callers that cannot allocate)
against fhs_evaluate, through the C ABI (collected last: a failure here
hides nothing else): two calls in a row on each workload,
the second with fewer outputs, so that the static scratch holds the first
call's contents when the second starts.  Counts bit-exact, amplitudes within
1e-12 (the same kernels; the no-alloc call may batch the output pairs
differently to fit its scratch)."""
import numpy as np
import pytest

import workloads as w

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2608_01467_amd as fhs  # noqa: E402

TOL = 1e-12


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return fhs.Context(0)


def _host(amps, stats):
    torch.cuda.synchronize()
    a = amps.cpu().numpy()
    return a[:, 0] + 1j * a[:, 1], stats.cpu().numpy().view(np.uint64)


def _both(ctx, inputs, coeffs, outputs, thr):
    ref = _host(*ctx.evaluate(inputs, coeffs, outputs, threshold=thr))
    # outputs pre-filled with garbage: the call must write every entry
    M = len(outputs)
    amps = torch.full((M, 2), float("nan"), dtype=torch.float64, device="cuda:0")
    stats = torch.full((M, 4), -1, dtype=torch.int64, device="cuda:0")
    got = _host(*ctx.evaluate_noalloc(inputs, coeffs, outputs, threshold=thr, out=(amps, stats)))
    return ref, got


def _assert_same(ref, got, what):
    assert np.abs(ref[0] - got[0]).max() <= TOL, what
    assert np.array_equal(ref[1][:, :3], got[1][:, :3]), what
    assert np.array_equal(ref[1][:, 3], got[1][:, 3]), what


@pytest.mark.parametrize("case", ["walk", "qaoa", "qaoa_pruned", "qft"])
def test_noalloc_matches_evaluate(ctx, case):
    thr = 0.0
    if case == "walk":
        # one batch, compiled consumer cached by the evaluate call before it
        cfg = w.CONFIGS["walk_99p_20s"]()
        part, launch = (1989, 2785), (2, 256, 0, 3)
        sizes = (8192, 1024)
    elif case.startswith("qaoa"):
        # the prefix table (2^17 entries per pair) spills the scratch: many batches
        cfg = w.CONFIGS["qaoa_12v_p2"]()
        part, launch = (35, 40), (2, 256, 0, 3)
        sizes = (512, 96)
        thr = 1e-6 if case == "qaoa_pruned" else 0.0
    else:
        cfg = w.CONFIGS["qft_20q"]()      # no sources: precheck and reductions only
        part, launch = (0, 0), (0, 0, 0, 0)
        sizes = (256, 17)
    prog = fhs.Program(cfg["circuit"].to_text())
    ctx.set_launch_config(*launch)
    ctx.load(prog)
    ctx.set_partition(*part)
    coeffs = [complex(*z) for z in cfg["coeffs"]]
    for m in sizes:
        ref, got = _both(ctx, cfg["inputs"], coeffs, cfg["outputs"][:m], thr)
        _assert_same(ref, got, (case, m))
    ctx.set_launch_config(0, 0, 0, 0)


def test_noalloc_too_large(ctx):
    """One pair's prefix table larger than the scratch: FHS_ENOMEM, detected
    before any launch, outputs untouched."""
    cfg = w.CONFIGS["qaoa_12v_p2"]()
    prog = fhs.Program(cfg["circuit"].to_text())
    ctx.load(prog)
    ctx.set_partition(prog.G, prog.G)      # every source in the prefix: 2^24 entries per pair
    amps = torch.zeros((2, 2), dtype=torch.float64, device="cuda:0")
    stats = torch.zeros((2, 4), dtype=torch.int64, device="cuda:0")
    with pytest.raises(fhs.FhsError) as ei:
        ctx.evaluate_noalloc([0], [1], [1, 2], out=(amps, stats))
    assert ei.value.status == 4
    torch.cuda.synchronize()
    assert (amps == 0).all() and (stats == 0).all()
