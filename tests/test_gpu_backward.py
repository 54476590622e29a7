"""GPU adjoint (gh_backward through torch.autograd) against the oracle's FP64
analytic adjoint, which is itself pinned to central differences.

Loss: mean squared distance of the mesh vertices to their nearest target on
a radius-0.4 sphere (nearest targets held fixed).  The forward is FP32; the
bar is ||g_gpu - g_oracle|| <= 1e-3 ||g_oracle||.
"""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint as oadj
from oracle import hop as ohop
from oracle import sdb as osdb

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _gpu_grad(torch, net, n, lo, h, targets, precision="fp32", margin=0.0):
    from paper_2111_05778_amd.autograd import GridHopMesh, flatten
    theta = torch.tensor(flatten(net), device="cuda", requires_grad=True)
    V = GridHopMesh.apply(theta, net, n, float(lo), float(h), precision, margin)
    Q = torch.tensor(targets, device="cuda", dtype=torch.float32)
    with torch.no_grad():
        nearest = torch.cdist(V, Q).argmin(dim=1)
    L = ((V - Q[nearest]) ** 2).sum(dim=1).mean()
    L.backward()
    return float(L.detach()), theta.grad.detach().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("width,n", [(64, 48), (256, 64)])
def test_gradient_matches_oracle_adjoint(torch_mod, width, n):
    net = W.neural_scene(0, width)
    g = W.grid(n)
    targets = W.loss_targets().astype(np.float64)
    L, grad = _gpu_grad(torch_mod, net, *g, targets)
    mesh = ohop.gridhop(osdb.SDB.neural(net), *g).mesh
    Lo, go, _ = oadj.adjoint(net, mesh, targets)
    rel = np.linalg.norm(grad - go) / np.linalg.norm(go)
    print(f"width {width} n {n}: L gpu {L:.6e} oracle {Lo:.6e}, |g| {np.linalg.norm(go):.3e}, rel err {rel:.2e}",
          flush=True)
    assert abs(L - Lo) <= 1e-5 * Lo
    assert rel <= 1e-3


def test_full_size_backward_n256(torch_mod):
    # the backward workload: width 256, N = 256, FP32 forward
    net = W.neural_scene(0, 256)
    g = W.grid(256)
    targets = W.loss_targets().astype(np.float64)
    L, grad = _gpu_grad(torch_mod, net, *g, targets)
    mesh = ohop.gridhop(osdb.SDB.neural(net), *g).mesh
    Lo, go, _ = oadj.adjoint(net, mesh, targets)
    rel = np.linalg.norm(grad - go) / np.linalg.norm(go)
    print(f"N=256 width 256: L gpu {L:.6e} oracle {Lo:.6e}, rel err {rel:.2e}", flush=True)
    assert rel <= 1e-3


def test_backward_is_deterministic(torch_mod):
    net = W.neural_scene(0, 128)
    g = W.grid(40)
    targets = W.loss_targets().astype(np.float64)
    _, a = _gpu_grad(torch_mod, net, *g, targets)
    _, b = _gpu_grad(torch_mod, net, *g, targets)
    np.testing.assert_array_equal(a, b)
