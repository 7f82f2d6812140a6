"""dpd_gradient_noalloc (the gradient with its scratch in the library's static
per-GPU array, no device allocation) against dpd_gradient: the same result
bit for bit on two calls in a row, the second on a smaller mesh, and with
muscle actuation; a mesh beyond the array's 16384 elements is rejected."""
import numpy as np
import pytest
import torch

import workloads as W
from parity_helpers import elem_dev, robot_scene

pytestmark = pytest.mark.gpu


def _inputs(mesh, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    X = mesh.rest_positions()
    x = X + 1e-3 * torch.randn(X.shape, generator=g, dtype=torch.float64).to(X.device)
    y = X + 1e-3 * torch.randn(X.shape, generator=g, dtype=torch.float64).to(X.device)
    return x, y


def test_noalloc_gradient_equals_gradient():
    from paper_2101_05917_amd.mesh import Mesh
    meshes = [Mesh.from_scene(W.config("c2")),                               # 1024 elements
              Mesh.from_scene(W.cantilever(3, 2, 2, youngs="loguniform", seed=5))]   # 12 elements
    for k, mesh in enumerate(meshes):
        x, y = _inputs(mesh, k)
        out = torch.full_like(x, float("nan"))
        got = mesh.gradient_noalloc(x, y, out=out)
        ref = mesh.gradient(x, y)
        torch.cuda.synchronize()
        print("mesh", k, "elements", mesh.n_elements, "|grad|", float(ref.norm()), flush=True)
        assert got.data_ptr() == out.data_ptr()
        assert torch.equal(got, ref)
    # muscle actuation and ground contact (the legged test body), after the two above
    sc = robot_scene()
    mesh = Mesh.from_scene(sc)
    x, y = _inputs(mesh, 7)
    act = elem_dev(np.random.default_rng(3).uniform(0.0, 1.0, mesh.n_elements))
    got = mesh.gradient_noalloc(x, y, act)
    ref = mesh.gradient(x, y, act)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    for m in meshes + [mesh]:
        m.close()


def test_noalloc_rejects_meshes_beyond_its_scratch():
    from paper_2101_05917_amd import _lib as L
    from paper_2101_05917_amd.mesh import Mesh
    sc = W.dropped_block(26, 26, 26, steps=1)          # 17576 elements
    mesh = Mesh.from_scene(sc, factorize=False)
    X = mesh.rest_positions()
    out = torch.zeros_like(X)
    with pytest.raises(L.DiffPDError) as e:
        mesh.gradient_noalloc(X, X, out=out)
    assert e.value.code == -1 and "16384" in str(e.value)
    torch.cuda.synchronize()
    assert torch.count_nonzero(out) == 0
    mesh.close()
