"""Differentiable internal force: ``internal_force(mesh, q, qdot, params)``.

Forward is the HIP f_int kernel; backward is the hand-written VJP kernel
(``tlfea_internal_force_vjp``), giving gradients with respect to q, qdot and the
material vector params = (p0, p1, p2, kv_eta, kv_lambda), where
(p0, p1, p2) = (E, nu, -) for SVK and (mu10, mu01, kappa) for Mooney-Rivlin.
"""
from __future__ import annotations

import torch

from .api import TLMesh
from .workloads import Material


class InternalForce(torch.autograd.Function):
    """Forward and backward read the material vector on the device
    (tlfea_internal_force_p / tlfea_internal_force_vjp_p): no host
    synchronisation, and the mesh's own material is left as it was."""

    @staticmethod
    def forward(ctx, mesh: TLMesh, q, qdot, params):
        p = params.detach().to(device=q.device, dtype=torch.float64).contiguous()
        f = mesh.internal_force_p(q.detach(), None if qdot is None else qdot.detach(), p)
        ctx.mesh = mesh
        ctx.has_qdot = qdot is not None
        ctx.save_for_backward(q, qdot if qdot is not None else torch.zeros_like(q), p)
        return f

    @staticmethod
    def backward(ctx, grad_f):
        q, qdot, p = ctx.saved_tensors
        mesh: TLMesh = ctx.mesh
        want_q, want_qd, want_p = ctx.needs_input_grad[1], ctx.needs_input_grad[2], ctx.needs_input_grad[3]
        want_qd = want_qd and ctx.has_qdot
        if not (want_q or want_qd or want_p):
            return None, None, None, None
        gq, gqd, gp = mesh.vjp_p(q.detach(), qdot.detach(), p, grad_f.contiguous().double(),
                                 want_q=want_q, want_qdot=want_qd, want_params=want_p)
        return None, gq, gqd, gp


def material_vector(material: Material, device) -> torch.Tensor:
    p = list(material.params) + [0.0] * (3 - len(material.params))
    return torch.tensor(p[:3] + [material.kv_eta, material.kv_lambda], dtype=torch.float64, device=device)


def internal_force(mesh: TLMesh, q, qdot=None, params=None):
    if params is None:
        params = material_vector(mesh.material, q.device)
    return InternalForce.apply(mesh, q, qdot, params)
