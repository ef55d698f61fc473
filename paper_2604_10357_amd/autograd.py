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
    @staticmethod
    def forward(ctx, mesh: TLMesh, q, qdot, params):
        vals = params.detach().double().cpu().tolist()
        mat = Material(mesh.material.kind, tuple(vals[:3]), vals[3], vals[4])
        mesh.set_material(mat)
        f = mesh.internal_force(q.detach(), None if qdot is None else qdot.detach())
        ctx.mesh = mesh
        ctx.mat = mat
        ctx.save_for_backward(q, qdot if qdot is not None else torch.zeros_like(q))
        ctx.has_qdot = qdot is not None
        return f

    @staticmethod
    def backward(ctx, grad_f):
        q, qdot = ctx.saved_tensors
        mesh: TLMesh = ctx.mesh
        mesh.set_material(ctx.mat)
        want_q, want_qd, want_p = ctx.needs_input_grad[1], ctx.needs_input_grad[2], ctx.needs_input_grad[3]
        gq, gqd, gp = mesh.vjp(q.detach(), qdot.detach(), grad_f.contiguous().double(),
                               want_q=want_q or True, want_qdot=want_qd and ctx.has_qdot, want_params=want_p)
        return None, (gq if want_q else None), (gqd if want_qd and ctx.has_qdot else None), gp


def material_vector(material: Material, device) -> torch.Tensor:
    p = list(material.params) + [0.0] * (3 - len(material.params))
    return torch.tensor(p[:3] + [material.kv_eta, material.kv_lambda], dtype=torch.float64, device=device)


def internal_force(mesh: TLMesh, q, qdot=None, params=None):
    if params is None:
        params = material_vector(mesh.material, q.device)
    return InternalForce.apply(mesh, q, qdot, params)
