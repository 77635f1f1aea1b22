"""The allocator hook of the C ABI (bem_set_allocator) with PyTorch's caching
allocator behind it: a mesh built through it gives bit-identical operator
applications and solves to one built on hipMalloc, its plan memory shows up in
torch's allocated bytes while it lives and goes back when it is destroyed,
and meshes built before and after the switch keep working side by side."""

import numpy as np
import pytest

import synth
from gpu_util import to_dev, to_host, announce

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bem():
    from paper_2312_00005_amd import bemfmm
    return bemfmm


def test_torch_allocator_backs_plan_memory(bem):
    import torch
    announce("allocator hook: torch caching allocator vs hipMalloc, ico4 tight 3-level FMM")
    nodes, tris = synth.icosphere(4)
    N = len(tris)
    k = 2 * np.pi / (6.0 * synth.mean_edge_length(nodes, tris))
    x = to_dev(synth.complex_normal(N, seed=4))
    ref_mesh = bem.Mesh(nodes, tris, "tight", use_fmm=1, levels=3, leaf_size=32)
    ref_mesh.set_problem(k)
    y_ref = to_host(ref_mesh.apply(x))
    p_ref, _, _ = ref_mesh.solve(ref_mesh.rhs_plane_wave())
    p_ref = to_host(p_ref)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    bem.use_torch_allocator()
    try:
        m = bem.Mesh(nodes, tris, "tight", use_fmm=1, levels=3, leaf_size=32)
        m.set_problem(k)
        y = to_host(m.apply(x))
        p, _, _ = m.solve(m.rhs_plane_wave())
        p = to_host(p)
        torch.cuda.synchronize()
        held = torch.cuda.memory_allocated() - before
        ws = m.workspace_bytes()
        announce(f"  torch holds {held / 2**20:.1f} MiB for the mesh, workspace {ws / 2**20:.1f} MiB")
        assert np.array_equal(y, y_ref)
        assert np.array_equal(p, p_ref)
        # the mesh's buffers (plus the solve's outputs) are torch's now
        assert held >= 0.9 * ws
        # the mesh built on hipMalloc still works beside it
        assert np.array_equal(to_host(ref_mesh.apply(x)), y_ref)
        del p
        m.close()
        torch.cuda.synchronize()
        after = torch.cuda.memory_allocated() - before
        announce(f"  after destroy: {after / 2**20:.2f} MiB")
        assert after < 0.01 * ws + 2**20
    finally:
        bem.use_hip_allocator()
    # and hipMalloc again for new meshes
    m2 = bem.Mesh(nodes, tris, "tight", use_fmm=1, levels=3, leaf_size=32)
    m2.set_problem(k)
    assert np.array_equal(to_host(m2.apply(x)), y_ref)
