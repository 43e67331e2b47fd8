"""The 256-problem batched workload against the oracle: M, N, K each
log-uniform in [256, 6144] and rounded to multiples of 64 (shape seed 3001),
entries uniform[-1, 1) from the seeded generator, device-resident, one
fastmm_gemm_batched call.  It runs with an explicit depth (leaf cutoff 128,
so every problem takes at least one Winograd level) and with each planner
mode choosing every problem's depth and tile.  Every problem is checked
against the FP64-accumulated classic product on 4 sampled rows (exact FP64
rows) and by Freivalds' check (C x against A (B x) for a +-1 vector x), each
within the Winograd tolerance 1e-4 of relative error."""
import numpy as np
import pytest

import synthgen
from oracle import checks
from tests.gpu_util import say

pytestmark = pytest.mark.gpu

TOL = 1e-4
COUNT = 256


@pytest.fixture(scope="module")
def workload(fastmm):
    import torch
    shapes = [tuple(int(v) for v in s) for s in synthgen.shapes_loguniform(3001, COUNT, lo=256, hi=6144)]
    say(f"batched workload: {COUNT} problems, generating operands")
    hA, hB, As, Bs, Cs = [], [], [], [], []
    for i, (m, n, k) in enumerate(shapes):
        sa, sb = synthgen.batch_seeds(5, i)
        a = synthgen.uniform_pm1(sa, m, k)
        b = synthgen.uniform_pm1(sb, k, n)
        hA.append(a)
        hB.append(b)
        As.append(torch.from_numpy(a).to("cuda"))
        Bs.append(torch.from_numpy(b).to("cuda"))
        Cs.append(torch.empty((m, n), dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    return shapes, hA, hB, As, Bs, Cs


def _check_all(shapes, hA, hB, Cs, tag):
    worst_s, worst_f = 0.0, 0.0
    for i, (m, n, k) in enumerate(shapes):
        C = Cs[i].cpu().numpy()
        assert np.isfinite(C).all(), f"{tag}: problem {i} has non-finite entries"
        rows = synthgen.row_sample(7100 + i, m, 4)
        es = checks.sampled_rows_rel(C, hA[i], hB[i], rows)
        ef = checks.freivalds_rel(C, hA[i], hB[i], synthgen.signs_pm1(7400 + i, n))
        assert es <= TOL and ef <= TOL, f"{tag}: problem {i} {m}x{n}x{k}: rows {es:.2e} freivalds {ef:.2e}"
        worst_s, worst_f = max(worst_s, es), max(worst_f, ef)
    say(f"  {tag}: worst sampled-rows {worst_s:.2e}, worst Freivalds {worst_f:.2e}")


def _fill_nan(Cs):
    for C in Cs:
        C.fill_(float("nan"))


def test_workload_explicit_depth(fastmm, workload):
    shapes, hA, hB, As, Bs, Cs = workload
    _fill_nan(Cs)
    say("batched workload: depth 3, leaf cutoff 128")
    fastmm.gemm_batched(As, Bs, Cs, depth=[3] * COUNT, leaf=[128] * COUNT)
    st = fastmm.get_stats()
    # every problem splits at least once; the largest three times
    assert st["depth"] == 3
    assert st["leaves"] >= 7 * COUNT
    _check_all(shapes, hA, hB, Cs, "explicit depth")
    # a replay of the captured graph on the same buffers gives the same bits
    first = [C.cpu().numpy() for C in Cs[:16]]
    fastmm.gemm_batched(As, Bs, Cs, depth=[3] * COUNT, leaf=[128] * COUNT)
    assert fastmm.get_stats()["graph_replayed"] == 1
    for a, C in zip(first, Cs[:16]):
        assert np.array_equal(a, C.cpu().numpy())


@pytest.mark.parametrize("mode", ["default", "model", "exhaustive"])
def test_workload_planner_modes(fastmm, workload, mode, request):
    shapes, hA, hB, As, Bs, Cs = workload
    if mode == "model":
        request.getfixturevalue("trained_planner")
    code = {"default": fastmm.PLAN_DEFAULT, "model": fastmm.PLAN_MODEL,
            "exhaustive": fastmm.PLAN_EXHAUSTIVE}[mode]
    fastmm.set_plan_mode(code)
    try:
        _fill_nan(Cs)
        say(f"batched workload: planner mode {mode}")
        fastmm.gemm_batched(As, Bs, Cs)
        st = fastmm.get_stats()
        say(f"  depth {st['depth']} leaves {st['leaves']} launches {st['launches']}")
        _check_all(shapes, hA, hB, Cs, mode)
    finally:
        fastmm.set_plan_mode(fastmm.PLAN_DEFAULT)
