"""torch.autograd wrappers: forward and backward both run the library's
hand-written kernels (the backward calls the "_bwd" entry points, which
recompute the forward pass from the saved inputs instead of storing
intermediates)."""

import torch

from . import glv


class InvariantMass(torch.autograd.Function):
    @staticmethod
    def forward(ctx, coords, mode, *cols):
        a, b = cols[:4], cols[4:]
        ctx.coords, ctx.mode = coords, mode
        ctx.save_for_backward(*cols)
        return glv.glv_invariant_mass(a, b, coords=coords, mode=mode)

    @staticmethod
    def backward(ctx, gm):
        cols = ctx.saved_tensors
        if ctx.mode == "compensated":  # the reverse mode of the cancellation-free form
            ga, gb = glv.glv_invariant_mass_comp_bwd(cols[:4], cols[4:], gm.contiguous())
        else:
            ga, gb = glv.glv_invariant_mass_bwd(cols[:4], cols[4:], gm.contiguous(), coords=ctx.coords)
        return (None, None) + tuple(ga) + tuple(gb)


class Boost(torch.autograd.Function):
    @staticmethod
    def forward(ctx, *cols):
        x, beta = cols[:4], cols[4:]
        ctx.save_for_backward(*cols)
        return glv.glv_boost(x, beta)

    @staticmethod
    def backward(ctx, *gy):
        cols = ctx.saved_tensors
        x, beta = cols[:4], cols[4:]
        gy = tuple(g.contiguous() if g is not None else torch.zeros_like(x[0]) for g in gy)
        per_item = beta[0].numel() == x[0].numel()
        gx, gbeta = glv.glv_boost_bwd(x, beta, gy, want_beta=per_item and any(ctx.needs_input_grad[4:]))
        if gbeta is None:
            gbeta = (None, None, None)
        return tuple(gx) + tuple(gbeta)


class EventReduce(torch.autograd.Function):
    """(total (4), event_m, pair_m) of CSR events; differentiable w.r.t. the
    particle columns (plain mode)."""

    @staticmethod
    def forward(ctx, offsets, pair_offsets, coords, *p):
        total, em, pm = glv.glv_event_reduce(p, offsets, pair_offsets, coords=coords, mode="plain")
        ctx.coords = coords
        ctx.save_for_backward(offsets, pair_offsets, *p)
        return (*total, em, pm)

    @staticmethod
    def backward(ctx, g0, g1, g2, g3, gem, gpm):
        offsets, pair_offsets, *p = ctx.saved_tensors
        ne = offsets.numel() - 1
        gt = [g if g is not None else torch.zeros(ne, dtype=p[0].dtype, device=p[0].device) for g in (g0, g1, g2, g3)]
        gp = glv.glv_event_reduce_bwd(p, offsets, pair_offsets, grad_total=[g.contiguous() for g in gt],
                                      grad_event_m=gem.contiguous() if gem is not None else None,
                                      grad_pair_m=gpm.contiguous() if gpm is not None else None, coords=ctx.coords)
        return (None, None, None) + tuple(gp)


def invariant_mass(a, b, coords="PtEtaPhiM", mode="plain"):
    """Differentiable pair mass of two 4-column legs."""
    return InvariantMass.apply(coords, mode, *a, *b)


def boost(x, beta):
    """Differentiable boost of (px, py, pz, E) columns by beta columns.

    beta holds one velocity per vector or one for all (single-element
    columns).  A broadcast beta gets no gradient (it would be a sum over all
    items, a reduction rather than an element-wise step), so a broadcast beta
    that requires one is rejected with ValueError."""
    if beta[0].numel() != x[0].numel() and any(b.requires_grad for b in beta):
        raise ValueError("boost: a broadcast beta (one velocity for all vectors) has no gradient; "
                         "pass one velocity per vector or detach beta")
    return Boost.apply(*x, *beta)


def event_reduce(p, offsets, pair_offsets=None, coords="PtEtaPhiM"):
    if pair_offsets is None:
        pair_offsets = glv.glv_pair_offsets(offsets)
    out = EventReduce.apply(offsets, pair_offsets, coords, *p)
    return tuple(out[:4]), out[4], out[5]


def _grads(gy, like):
    return tuple(g.contiguous() if g is not None else torch.zeros_like(like) for g in gy)


class Convert(torch.autograd.Function):
    @staticmethod
    def forward(ctx, src, dst, *cols):
        ctx.src, ctx.dst = src, dst
        ctx.save_for_backward(*cols)
        return glv.glv_convert(cols, src, dst)

    @staticmethod
    def backward(ctx, *gy):
        cols = ctx.saved_tensors
        return (None, None) + tuple(glv.glv_convert_bwd(cols, _grads(gy, cols[0]), ctx.src, ctx.dst))


class LorentzTransform(torch.autograd.Function):
    """y = L x (or a Rotation3D); differentiable w.r.t. x and, for one matrix
    per item, the matrix (a broadcast matrix gets no gradient)."""

    @staticmethod
    def forward(ctx, kind, *cols):
        x, m = cols[:4], cols[4:]
        ctx.kind = kind
        ctx.save_for_backward(*cols)
        fn = glv.glv_lorentz_transform if kind == "lorentz" else glv.glv_rotate
        return fn(x, m)

    @staticmethod
    def backward(ctx, *gy):
        cols = ctx.saved_tensors
        x, m = cols[:4], cols[4:]
        per_item = m[0].numel() == x[0].numel()
        fn = glv.glv_lorentz_transform_bwd if ctx.kind == "lorentz" else glv.glv_rotate_bwd
        gx, gm = fn(x, m, _grads(gy, x[0]), want_matrix=per_item and any(ctx.needs_input_grad[5:]))
        return (None,) + tuple(gx) + (tuple(gm) if gm is not None else (None,) * len(m))


class RotateAxisAngle(torch.autograd.Function):
    """Differentiable w.r.t. the vectors only (not the axis and angle)."""

    @staticmethod
    def forward(ctx, *cols):
        x, aa = cols[:4], cols[4:]
        ctx.save_for_backward(x[0], *aa)
        return glv.glv_rotate_axis_angle(x, aa)

    @staticmethod
    def backward(ctx, *gy):
        x0, *aa = ctx.saved_tensors
        return tuple(glv.glv_rotate_axis_angle_bwd(aa, _grads(gy, x0))) + (None,) * 4


def convert(cols, src, dst):
    """Differentiable coordinate conversion of 4 columns from ``src`` to ``dst``."""
    return Convert.apply(src, dst, *cols)


def lorentz_transform(x, L):
    """Differentiable y = L x (L: 16 row-major columns, per item or broadcast)."""
    return LorentzTransform.apply("lorentz", *x, *L)


def rotate(x, R):
    """Differentiable Rotation3D of (px, py, pz) (R: 9 row-major columns)."""
    return LorentzTransform.apply("rotate", *x, *R)


def rotate_axis_angle(x, axis_angle):
    """AxisAngle rotation, differentiable w.r.t. x (the axis and angle are
    treated as constants)."""
    return RotateAxisAngle.apply(*x, *axis_angle)
