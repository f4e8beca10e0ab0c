"""Host-side checks of the checkpoint planner (no GPU): the memory accounting and the
choice of the shallowest nesting that fits a budget."""
import pytest

from paper_2605_26677_amd.rollout import checkpoint_plan, memory_model


def test_every_k_accounting():
    """Every-K at 512^2 FP32: floor(N/K) + 1 snapshot pairs (96 + 24 B per node) and
    K + 1 records (24 B per node)."""
    n, N, K = 512, 2000, 100
    m = memory_model(n, n, "f32", N, [K])
    nodes = n * n
    assert m["snapshots"] == (N // K + 1) * 120 * nodes
    assert m["records"] == (K + 1) * 24 * nodes
    assert m["forward_passes"] == 2


def test_nesting_trades_memory_for_replays():
    n, N = 4096, 20000
    flat = memory_model(n, n, "f32", N, [141])
    nested = memory_model(n, n, "f32", N, [2000, 100])
    assert nested["peak"] < flat["peak"] and nested["forward_passes"] == flat["forward_passes"] + 1


@pytest.mark.parametrize("budget_gib", [64, 96, 128, 256])
def test_plan_fits_budget_with_fewest_levels(budget_gib):
    n, N = 4096, 20000
    B = budget_gib * 2 ** 30
    K = checkpoint_plan(n, n, "f32", N, B)
    assert memory_model(n, n, "f32", N, K)["peak"] <= B
    assert all(a > b for a, b in zip(K, K[1:]))
    if len(K) > 1:
        # one level fewer does not fit at any split the planner considers
        with pytest.raises(ValueError):
            checkpoint_plan(n, n, "f32", N, B, max_depth=len(K) - 1)


def test_plan_refuses_impossible_budget():
    with pytest.raises(ValueError):
        checkpoint_plan(4096, 4096, "f32", 20000, 8 * 2 ** 30)


def test_host_top_level_cuts_replays_within_budgets():
    """With the outermost snapshots in pinned host memory the 4096^2 x 20000 FP32 adjoint
    fits 64 GiB of device memory with two levels (three forward passes) instead of four."""
    from paper_2605_26677_amd.rollout import plan_checkpoints
    n, N = 4096, 20000
    dev, host = 64 * 2 ** 30, 48 * 2 ** 30
    flat = plan_checkpoints(n, n, "f32", N, dev)
    with_host = plan_checkpoints(n, n, "f32", N, dev, host)
    assert not flat["host_top"] and with_host["host_top"]
    assert with_host["model"]["forward_passes"] < flat["model"]["forward_passes"]
    assert with_host["model"]["peak"] <= dev and with_host["model"]["host"] <= host
    m = memory_model(n, n, "f32", N, with_host["levels"], host_top=True)
    assert m["host"] == (N // with_host["levels"][0] + 1) * (96 + 24) * n * n


@pytest.mark.parametrize("bad", [[-1, 3], [0, 64], [5, 4096]])
def test_rollout_rejects_probes_outside_the_grid(bad):
    """Probe indices reach device memory in the adjoint kernels; RolloutConfig rejects any
    outside [0, nx*ny) before a GPU is touched (an 8 x 8 grid has nodes 0..63)."""
    import torch
    from paper_2605_26677_amd.rollout import RolloutConfig
    with pytest.raises(ValueError):
        RolloutConfig(nx=8, ny=8, c=2.0, omega=2.0, nsteps=4, probes=torch.tensor(bad))


def test_rollout_probe_dtype_and_shape():
    import torch
    from paper_2605_26677_amd.rollout import RolloutConfig
    with pytest.raises(ValueError):
        RolloutConfig(nx=8, ny=8, c=2.0, omega=2.0, nsteps=4, probes=torch.tensor([1.0, 2.0]))
    with pytest.raises(ValueError):
        RolloutConfig(nx=8, ny=8, c=2.0, omega=2.0, nsteps=4, probes=torch.tensor([[1, 2]]))
    cfg = RolloutConfig(nx=8, ny=8, c=2.0, omega=2.0, nsteps=4, probes=torch.tensor([0, 63]))
    assert cfg.probes.numel() == 2
