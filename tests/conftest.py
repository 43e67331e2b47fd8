import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def fastmm():
    """The GPU library binding.  On a machine with a GPU a missing build is an error,
    never a skip: the tests must exercise the native library."""
    from paper_1205_2927_amd import fastmm as fm
    fm.load()
    return fm


# Planner training set: 160 shapes, M, N, K log-uniform in [256, 6144] in
# multiples of 64 (the distribution of the batched workload), seed 4001 --
# disjoint from the evaluation shapes (seed 3001).
PLANNER_TRAIN_SHAPES = 160


@pytest.fixture(scope="session")
def trained_planner(fastmm):
    """Times every candidate plan of the training shapes on the device
    (EXHAUSTIVE mode fills the timing database) and trains the cost model on
    the GPU.  Returns the final training loss."""
    import synthgen
    shapes = synthgen.shapes_loguniform(4001, PLANNER_TRAIN_SHAPES)
    print(f"planner: timing {len(shapes)} training shapes", flush=True)
    for i, (M, N, K) in enumerate(shapes):
        fastmm.plan(int(M), int(N), int(K), fastmm.PLAN_EXHAUSTIVE)
        if i % 40 == 39:
            print(f"  {i + 1} shapes, {fastmm.planner_records()} records", flush=True)
    loss = fastmm.planner_train(epochs=400, batch=64, lr=3e-3, seed=4001)
    print(f"planner: trained on {fastmm.planner_records()} records, loss {loss:.4f}", flush=True)
    return loss
