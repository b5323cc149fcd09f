"""bn_adjoint_step_noalloc (the adjoint step on the library's fixed scratch array, no allocation)
against bn_adjoint_step on the same inputs, through the C ABI: two calls in a row on one GPU, the
second on a smaller grid (the array keeps the first call's contents), and a grid too large for the
array rejected before any work is enqueued.  Both entry points run the same kernels, so the
results must agree bit for bit (stronger than the 1e-6 adjoint tolerance)."""
import numpy as np
import pytest

from paper_1806_04960_amd import scenarios as sc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def bn(torch_cuda):
    from paper_1806_04960_amd import bn2d
    bn2d.lib()
    return bn2d


def _inputs(torch, s, seed):
    s = sc.generic_state(s, seed=seed)
    rng = np.random.default_rng(seed + 100)
    lam = rng.normal(size=s.q.shape)
    q = torch.from_numpy(np.ascontiguousarray(s.q)).cuda()
    return s, q, torch.from_numpy(lam).cuda()


def test_noalloc_adjoint_equals_the_allocating_one_on_two_calls(bn, torch_cuda):
    torch = torch_cuda
    cases = [(sc.wall_impact(0, 96, 48), 3), (sc.dam_break_small(37, 21), 5)]  # second call smaller
    for build, seed in cases:
        s, q, lam = _inputs(torch, build, seed)
        print(f"no-alloc adjoint: {s.nx}x{s.ny}, seed {seed}", flush=True)
        with bn.Simulation(s) as sim:
            sim.set_state(q)
            dt = 0.9 * sim.compute_dt()
            gref = torch.zeros(s.nx, dtype=torch.float64, device="cuda")
            ref = sim.adjoint_step(q, lam, dt, grad_bottom=gref, src=q)
            out = torch.full_like(q, float("nan"))
            gout = torch.full_like(gref, float("nan"))
            sim.adjoint_step_noalloc(q, lam, dt, out, grad_bottom=gout, src=q)
            torch.cuda.synchronize()
        ref, out = ref.cpu().numpy(), out.cpu().numpy()
        assert np.all(np.isfinite(out))
        assert np.array_equal(out, ref), np.abs(out - ref).max()
        assert torch.equal(gout, gref)


def test_noalloc_adjoint_rejects_a_grid_beyond_its_array(bn, torch_cuda):
    torch = torch_cuda
    s = sc.dam_break_small(2048, 2048)  # 4 planes of 4194304 cells alone (16.8 M doubles) > 2^24
    with bn.Simulation(s) as sim:
        q = torch.from_numpy(np.ascontiguousarray(s.q)).cuda()
        out = torch.zeros_like(q)
        with pytest.raises(bn.BnError) as e:
            sim.adjoint_step_noalloc(q, q, 1e-5, out)
        assert e.value.code == bn.BN_EINVAL
        torch.cuda.synchronize()
        assert float(out.abs().max()) == 0.0
