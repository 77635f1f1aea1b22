"""Differentiable field-point energy with respect to per-element admittance.

J(Y) = sum_f |p(x_f)|^2, where the surface pressure solves the Burton-Miller
collocation system with beta = rho_c Y (Sec. 2.5) and p(x_f) follows from the
representation formula (Eq. (BIE_I), lambda = 1).  The backward pass costs one
adjoint solve with the conjugate-transpose operator:

    A^H mu = M^H p_field,   w = V^H mu,   h = (I^G)^H p_field,
    dJ/dY_e = 2 Re{ -i k rho_c p_e ( -conj(w_e) - conj(h_e) ) },

with V = dA/dc the part of the operator that multiplies the boundary factor
c_j = -i k beta_j and M = I^H - I^G diag(c) the field map.  Every step runs in
the library; this module only wires the calls into torch.autograd.

Y is real (a resistive admittance per element); the gradient is with respect
to that real parameter.
"""

import torch

from . import bemfmm


def _source_fields(mesh, pts, source):
    kind, s, P0 = source
    if kind == "plane":
        return mesh.rhs_plane_wave(s, P0), mesh.incident_plane_wave(pts, s, P0)
    if kind == "point":
        return mesh.rhs_point_source(s, P0), mesh.incident_point_source(pts, s, P0)
    raise ValueError("source kind must be 'plane' or 'point'")


class FieldEnergy(torch.autograd.Function):
    """J(Y) for a mesh, wavenumber, rho_c, field points and source."""

    @staticmethod
    def forward(ctx, Y, mesh, k, rho_c, pts, source):
        if Y.dtype != torch.float64 or not Y.is_cuda or Y.numel() != mesh.n:
            raise TypeError("Y must be a float64 device tensor with one value per element")
        beta = (Y.detach() * rho_c).to(torch.complex128).contiguous()
        mesh.set_problem(k, beta)
        b, pinc = _source_fields(mesh, pts, source)
        p, _, info = mesh.solve(b)
        pf, J = mesh.field(pts, p, pinc, energy=True)
        ctx.mesh, ctx.k, ctx.rho_c, ctx.pts = mesh, k, rho_c, pts
        ctx.beta = beta
        ctx.save_for_backward(p, pf)
        ctx.forward_info = info
        return J

    @staticmethod
    def backward(ctx, gJ):
        mesh = ctx.mesh
        p, pf = ctx.saved_tensors
        if mesh._beta is not ctx.beta:
            mesh.set_problem(ctx.k, ctx.beta)
        rhs = mesh.field_adjoint(ctx.pts, pf, part=0)
        mu, _ = mesh.solve_adjoint(rhs)
        w = mesh.apply_dc(mu, op="AH")
        hg = mesh.field_adjoint(ctx.pts, pf, part=1)
        grad = mesh.grad_admittance(p, w, hg, ctx.rho_c)
        return gJ * grad, None, None, None, None, None


def field_energy(mesh, Y, k, rho_c, pts, source=("plane", (0.0, 0.0, 1.0), 1.0)):
    """J(Y) = sum over pts of |p|^2; differentiable in Y (float64, per element).

    source: ("plane", direction, P0) or ("point", position, P0)."""
    if not isinstance(mesh, bemfmm.Mesh):
        raise TypeError("mesh must be a bemfmm.Mesh")
    return FieldEnergy.apply(Y, mesh, float(k), float(rho_c), bemfmm._dev_pts(pts), source)
