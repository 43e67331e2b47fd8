"""The learned planner: GPU network kernels against the FP64 oracle, the
exhaustive autotuner, and the trained model evaluated by its regret against
exhaustive timing and by what it gains over the fixed rule."""
import numpy as np
import pytest

import synthgen
from oracle import classic, checks, mlp
from tests.gpu_util import dev, host, say, uniform

pytestmark = pytest.mark.gpu


def _case(seed=901, batch=33):
    flat = synthgen.uniform_pm1_np(seed, 1, mlp.N_PARAMS)[0] * np.float32(0.3)
    X = synthgen.uniform_pm1_np(seed + 1, batch, mlp.D_IN)
    t = synthgen.uniform_pm1_np(seed + 2, 1, batch)[0]
    return flat.astype(np.float32), X, t


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("batch", [1, 33, 256])
def test_mlp_forward_backward_match_oracle(fastmm, batch):
    import torch
    flat, X, t = _case(batch=batch)
    y_ref, cache = mlp.forward(flat.astype(np.float64), X.astype(np.float64))
    g_ref = mlp.backward(flat.astype(np.float64), cache, y_ref, t.astype(np.float64))
    loss_ref = mlp.loss(y_ref, t)
    dp, dX, dt = dev(flat), dev(X), dev(t)
    y = torch.empty(batch, device="cuda")
    fastmm.mlp_forward(batch, dp, dX, y)
    assert rel(host(y), y_ref) < 1e-5
    g = torch.empty(mlp.N_PARAMS, device="cuda")
    loss = torch.empty(1, device="cuda")
    fastmm.mlp_backward(batch, dp, dX, dt, g, loss)
    gh = host(g).astype(np.float64)
    # per tensor (W1, b1, W2, b2, W3, b3)
    o = 0
    for name, shape in mlp.SHAPES:
        size = int(np.prod(shape))
        e = rel(gh[o:o + size], g_ref[o:o + size])
        say(f"  batch={batch} grad {name}: rel={e:.2e}")
        assert e < 1e-4, name
        o += size
    assert abs(float(host(loss)[0]) - loss_ref) <= 1e-5 * max(1.0, loss_ref)


def test_mlp_adam_matches_oracle(fastmm):
    import torch
    flat, X, t = _case(seed=911)
    g = synthgen.uniform_pm1_np(912, 1, mlp.N_PARAMS)[0]
    m = synthgen.uniform_pm1_np(913, 1, mlp.N_PARAMS)[0] * np.float32(0.1)
    v = np.abs(synthgen.uniform_pm1_np(914, 1, mlp.N_PARAMS)[0]) * np.float32(0.01)
    p_ref, m_ref, v_ref = mlp.adam_step(flat.astype(np.float64), g.astype(np.float64),
                                        m.astype(np.float64), v.astype(np.float64), 3, 1e-3)
    dp, dm, dv = dev(flat), dev(m), dev(v)
    fastmm.mlp_adam(dev(g), dp, dm, dv, 3, 1e-3)
    assert rel(host(dm), m_ref) < 1e-6
    assert rel(host(dv), v_ref) < 1e-6
    assert np.max(np.abs(host(dp) - p_ref)) < 1e-6


def test_default_rule(fastmm):
    # deepest split whose leaf stays >= 1280 in every dimension; 64x64 tiles
    # when the leaf launch would have fewer than 512 tiles of 128x128
    for n, d, t in [(19456, 3, 0), (16384, 3, 0), (10240, 3, 0), (8192, 2, 0), (5632, 2, 0),
                    (4096, 1, 0), (3072, 1, 0), (2560, 1, 0), (2048, 0, 3), (512, 0, 3)]:
        p = fastmm.plan(n, n, n, fastmm.PLAN_DEFAULT)
        assert (p.depth, p.leaf, p.tile, p.source) == (d, 1280, t, fastmm.PLAN_DEFAULT), n
    p = fastmm.plan(19456, 12288, 16384, fastmm.PLAN_DEFAULT)  # leaves 2432 x 1536 x 2048
    assert p.depth == 3


def test_exhaustive_model_regret_and_gain(fastmm, trained_planner, tmp_path):
    # The cost model is trained (conftest) on the exhaustive timings of 160
    # shapes of seed 4001; it is evaluated on 48 held-out shapes of seed 3001
    # against exhaustive timing of every candidate: its mean regret must not
    # exceed the fixed rule's, and its choices must be at least as fast as
    # the fixed rule's (geometric mean over the shapes).
    import json
    loss = trained_planner
    assert np.isfinite(loss) and loss < 0.5
    eval_shapes = synthgen.shapes_loguniform(3001, 48)
    db = tmp_path / "db.json"
    model = tmp_path / "model.bin"
    fastmm.planner_save(None, str(model))
    assert model.stat().st_size == 4 * fastmm.MODEL_NETS * fastmm.MLP_PARAMS
    regrets_model, regrets_default, gains = [], [], []
    for (M, N, K) in eval_shapes:
        M, N, K = int(M), int(N), int(K)
        best = fastmm.plan(M, N, K, fastmm.PLAN_EXHAUSTIVE)
        pm = fastmm.plan(M, N, K, fastmm.PLAN_MODEL)
        pd = fastmm.plan(M, N, K, fastmm.PLAN_DEFAULT)
        assert pm.source == fastmm.PLAN_MODEL
        fastmm.planner_save(str(db), None)
        with open(db) as f:
            recs = [r for r in json.load(f)["records"] if (r["M"], r["N"], r["K"]) == (M, N, K)]
        table = {(r["depth"], r["tile"]): r["ms"] for r in recs}
        t_best = table[(best.depth, best.tile)]
        t_model = table[(pm.depth, pm.tile)]
        t_default = table[(pd.depth, pd.tile)]
        regrets_model.append(t_model / t_best - 1)
        regrets_default.append(t_default / t_best - 1)
        gains.append(t_default / t_model)
        say(f"  {M}x{N}x{K}: best d{best.depth}t{best.tile} {t_best:.3f} ms, model d{pm.depth}t{pm.tile} "
            f"{t_model:.3f}, default d{pd.depth}t{pd.tile} {t_default:.3f}")
    rm, rd = float(np.mean(regrets_model)), float(np.mean(regrets_default))
    gain = float(np.exp(np.mean(np.log(gains))))
    say(f"mean regret model={rm:.4f} default={rd:.4f}; geo-mean gain over default={gain:.4f}")
    assert rm <= rd
    assert gain >= 1.0
    # the saved model reproduces the same choices after a reload
    choices = [(fastmm.plan(int(M), int(N), int(K), fastmm.PLAN_MODEL).depth,
                fastmm.plan(int(M), int(N), int(K), fastmm.PLAN_MODEL).tile) for (M, N, K) in eval_shapes[:8]]
    fastmm.planner_load(None, str(model))
    again = [(fastmm.plan(int(M), int(N), int(K), fastmm.PLAN_MODEL).depth,
              fastmm.plan(int(M), int(N), int(K), fastmm.PLAN_MODEL).tile) for (M, N, K) in eval_shapes[:8]]
    assert choices == again


def test_auto_depth_product_is_correct(fastmm):
    n = 1536
    A = uniform(921, n, n)
    B = uniform(922, n, n)
    import torch
    C = torch.empty((n, n), device="cuda")
    fastmm.set_plan_mode(fastmm.PLAN_DEFAULT)
    fastmm.gemm(n, n, n, dev(A), dev(B), C, depth=fastmm.AUTO)
    assert fastmm.get_stats()["depth"] == 0  # 1536 / 2 = 768 < 1280
    assert checks.rel_frob(host(C), classic.gemm(A, B)) < 1e-4


def test_auto_depth_host_operands(fastmm):
    # With host operands the automatic depth is 0 below a smallest extent of
    # 6656 (the transfers bound the call there), and the planner's depth
    # from it on; device operands keep the planner's depth.  The plain
    # product from host memory is the device-resident one bit for bit.
    import torch
    fastmm.set_plan_mode(fastmm.PLAN_DEFAULT)
    for n in (4096, 6656):
        say(f"auto depth, host operands, n={n}")
        A = uniform(931 + n, n, n)
        B = uniform(932 + n, n, n)
        Cp = torch.full((n, n), float("nan")).pin_memory()
        fastmm.gemm(n, n, n, torch.from_numpy(A).pin_memory(), torch.from_numpy(B).pin_memory(), Cp,
                    depth=fastmm.AUTO)
        planned = fastmm.plan(n, n, n, fastmm.PLAN_DEFAULT).depth
        got = fastmm.get_stats()["depth"]
        Cd = torch.empty((n, n), device="cuda")
        if n < 6656:
            assert planned >= 1 and got == 0
            fastmm.gemm(n, n, n, dev(A), dev(B), Cd, depth=fastmm.AUTO)
            assert fastmm.get_stats()["depth"] == planned
            fastmm.gemm(n, n, n, dev(A), dev(B), Cd, depth=0)
            assert np.array_equal(Cp.numpy(), host(Cd))
        else:
            assert got == planned >= 1
        rows = synthgen.row_sample(933, n, 8)
        assert checks.sampled_rows_rel(Cp.numpy(), A, B, rows) <= 1e-4


def test_model_file_errors(fastmm, tmp_path):
    bad = tmp_path / "short.bin"
    bad.write_bytes(b"\0" * 100)
    with pytest.raises(fastmm.FastmmError) as e:
        fastmm.planner_load(None, str(bad))
    assert e.value.code == fastmm.ERROR_INVALID_VALUE
    nan = tmp_path / "nan.bin"
    nan.write_bytes(np.full(fastmm.MODEL_NETS * mlp.N_PARAMS, np.nan, np.float32).tobytes())
    with pytest.raises(fastmm.FastmmError):
        fastmm.planner_load(None, str(nan))
