"""The allocation-free adjoint entry point (srf_short_range_adjoint_noalloc)
against srf_short_range_adjoint, through the C ABI: two calls in a row on the
static workspace, the second with a smaller input, each equal to the
allocating entry point's result up to the order of its FP64 atomics; a tree
beyond the workspace is refused before anything is launched."""
import numpy as np
import pytest
import torch

import paper_1211_4406_amd as srf
import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def both(ps, seed, precision=srf.FP32_REL):
    p = srf.Params.of(ps.params, precision)
    x = torch.tensor(ps.positions(), dtype=torch.float64, device="cuda")
    m = torch.tensor(ps.m, dtype=torch.float64, device="cuda")
    w = torch.tensor(synth.loss_weights(ps.n, seed), dtype=torch.float64, device="cuda")
    tree = srf.tree_build(x, m, p)
    lists = srf.make_lists(tree, p)
    gx0, gm0 = srf.short_range_adjoint(tree, lists, p, w)
    gx = torch.full_like(gx0, float("nan"))
    gm = torch.full_like(gm0, float("nan"))
    srf.short_range_adjoint_noalloc(tree, lists, p, w, gx, gm)
    torch.cuda.synchronize()
    return gx0, gm0, gx, gm, (tree, lists, p, w)


def close(a, b):
    # the two paths run the same kernels; their FP64 atomics may add in
    # another order, so the results agree to FP64 rounding of the sums
    return torch.allclose(a, b, rtol=1e-12, atol=1e-12 * b.abs().max().item())


def test_noalloc_adjoint_matches_the_allocating_one_twice_in_a_row():
    big = synth.small_clustered(150_000, 401, r_cut=0.04, eps=2e-4, theta=0.5, per_halo=1500)
    small = synth.small_clustered(9_000, 402, r_cut=0.1, eps=2e-4, theta=0.5, per_halo=900)
    for ps, seed in ((big, 403), (small, 404)):
        say(f"[gpu] noalloc adjoint n={ps.n}")
        gx0, gm0, gx, gm, _ = both(ps, seed)
        assert torch.isfinite(gx).all() and torch.isfinite(gm).all()
        assert close(gx, gx0) and close(gm, gm0)
    say("[gpu] noalloc adjoint fp64, and no device allocation by the call")
    gx0, gm0, gx, gm, (tree, lists, p, w) = both(small, 405, srf.FP64)
    assert close(gx, gx0) and close(gm, gm0)
    free0, _ = torch.cuda.mem_get_info()
    for _ in range(3):
        srf.short_range_adjoint_noalloc(tree, lists, p, w, gx, gm)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 >= free0
    assert close(gx, gx0) and close(gm, gm0)


def test_noalloc_adjoint_refuses_a_tree_beyond_its_workspace():
    n = 2_600_000
    ps = synth.small_uniform(n, 406, r_cut=0.01, eps=1e-4, theta=0.5)
    p = srf.Params.of(ps.params)
    say(f"[gpu] noalloc adjoint beyond the workspace, n={n}")
    x = torch.tensor(ps.positions(), dtype=torch.float64, device="cuda")
    m = torch.tensor(ps.m, dtype=torch.float64, device="cuda")
    w = torch.ones((n, 3), dtype=torch.float64, device="cuda")
    tree = srf.tree_build(x, m, p)
    lists = srf.make_lists(tree, p)
    gx = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
    gm = torch.zeros((n,), dtype=torch.float64, device="cuda")
    with pytest.raises(srf.SrfError) as e:
        srf.short_range_adjoint_noalloc(tree, lists, p, w, gx, gm)
    assert e.value.status == -1 and "workspace" in str(e.value)
    torch.cuda.synchronize()
    assert bool((gx == 0).all()) and bool((gm == 0).all())
    info = tree.info()
    say(f"    n_cells={info['n_nodes']}, workspace needed {8 * (7 * n + 8 * info['n_nodes'])} B")
    assert np.isfinite(info["n_nodes"])
