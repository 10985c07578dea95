"""Algorithmic operation model of the contact-manifold path (per kept pair).

Counts the arithmetic the method itself requires, each step once: every
vertex-SDF candidate, every edge-edge pair's witness QP, witness SDF queries,
indicators and score, and the nearest-neighbour row / column LSE terms.  The
implementation's extra work (the max pass of the stable LSE, the recomputed
QP of the distance pass, the SoftSort pass over near-top candidates) is not
counted, so a roofline fraction built on this model is conservative.

Operation classes:
  fma   fused multiply-add (2 flops, one full-rate VALU slot)
  alu   other full-rate VALU op: add, mul, min/max, compare/select (1 flop)
  trans exp, log, reciprocal, division, sqrt (1 flop, a quarter-rate slot)
"""
from __future__ import annotations

import numpy as np

SPHERE, CAPSULE, BOX, POLYTOPE = 0, 1, 2, 3

# (fma, alu, trans) of one SDF query in the body frame
_SDF_ANALYTIC = {SPHERE: (2, 2, 2), CAPSULE: (2, 5, 2), BOX: (2, 16, 2)}
_XFORM = (9, 3, 0)             # pair frame -> body frame for the other body's queries
_GRAD_ROT = (9, 0, 0)          # gradient back to the pair frame


def sdf_cost(kind: int, nf: int, grad: bool, transformed: bool):
    """(fma, alu, trans) of one SDF value (+ gradient) query."""
    if kind == POLYTOPE:
        # per plane: 3 fma distance, 1 alu scale, 1 exp, 1 alu sum (+3 fma gradient)
        f, a, t = (3 + (3 if grad else 0)) * nf, 2 * nf, nf
        f, a, t = f, a + 2, t + 1 + (1 if grad else 0)      # log, (reciprocal)
    else:
        f, a, t = _SDF_ANALYTIC[kind]
        if grad:
            a += 3
    if transformed:
        f += _XFORM[0]; a += _XFORM[1]
        if grad:
            f += _GRAD_ROT[0]
    return np.array([f, a, t], dtype=np.int64)


# E-E per edge pair, excluding the SDF queries
_QP = np.array([30, 60, 26], dtype=np.int64)          # Q, c, det, alpha_u, 4 soft clips, 4 costs,
                                                      # soft argmin, 4 sigmoids + logs, blend, Delta e
_WITNESS = np.array([12, 6, 2], dtype=np.int64)       # e1, e2, |Delta e|, n_bar
_INDICATORS = np.array([9, 20, 10], dtype=np.int64)   # 2 soft signs, 3 log-sigmoids, dots, nn terms,
                                                      # two scores
_NN_LSE = np.array([0, 4, 2], dtype=np.int64)         # row + column LSE terms of D
# V-S per vertex, excluding the SDF query
_VS = np.array([3, 8, 4], dtype=np.int64)             # normal scaling, log-sigmoid, score


def pair_ops(kA: int, vA: int, eA: int, fA: int, kB: int, vB: int, eB: int, fB: int) -> np.ndarray:
    """(fma, alu, trans) of one kept pair (body A defines the pair frame)."""
    ops = np.zeros(3, dtype=np.int64)
    ops += vA * (sdf_cost(kB, fB, True, True) + _VS)
    ops += vB * (sdf_cost(kA, fA, True, False) + _VS)
    ee = (_QP + _WITNESS + _INDICATORS + _NN_LSE
          + sdf_cost(kB, fB, False, True) + sdf_cost(kA, fA, True, False)
          + sdf_cost(kA, fA, False, False) + sdf_cost(kB, fB, True, True))
    ops += eA * eB * ee
    return ops


def batch_ops(types, nv, ne, nf, pairs_a, pairs_b, body_geom) -> np.ndarray:
    """Summed (fma, alu, trans) over kept pairs; per-geometry arrays indexed by geometry id."""
    ga = body_geom[pairs_a]
    gb = body_geom[pairs_b]
    tot = np.zeros(3, dtype=np.int64)
    keys, counts = np.unique(np.stack([ga, gb]), axis=1, return_counts=True)
    for (x, y), c in zip(keys.T, counts):
        tot += c * pair_ops(types[x], nv[x], ne[x], nf[x], types[y], nv[y], ne[y], nf[y])
    return tot


def reverse_ops(forward: np.ndarray) -> np.ndarray:
    """(fma, alu, trans) of the reverse sweep of the vector-Jacobian product
    (cm_collide_backward), given the forward's count.

    Reverse-mode differentiation visits every forward operation once more:
    the adjoint of y = a b + c is a_bar += y_bar b, b_bar += y_bar a, c_bar +=
    y_bar (2 fma + 1 alu), of y = a op b for add / mul / compare-select at most
    2 alu, and of a transcendental y = f(x) one alu (x_bar += y_bar f'(x), with
    f' a multiple of y or of 1/x, both already computed).  So the sweep costs
    (2 fma, fma + 2 alu + trans, 0).  The forward recompute the adjoint kernel
    performs (it stores no E x E state) is implementation work and is not
    counted; the candidates whose SoftSort weights it drops as negligible are
    counted (the model counts every step of the definition once)."""
    fma, alu, trans = (int(x) for x in forward)
    return np.array([2 * fma, fma + 2 * alu + trans, 0], dtype=np.int64)


def _reverse(ops: np.ndarray) -> np.ndarray:
    """Reverse sweep of a forward count, as in reverse_ops (linear in the count)."""
    fma, alu, trans = (int(x) for x in ops)
    return np.array([2 * fma, fma + 2 * alu + trans, 0], dtype=np.int64)


def adjoint_pair_ops(kA: int, vA: int, eA: int, fA: int, kB: int, vB: int, eB: int, fB: int,
                     w_vsA: int, w_vsB: int, w_ee: int) -> np.ndarray:
    """(fma, alu, trans) the adjoint kernel's method does for one pair whose
    adjoint window (candidates within 18 tau of s_[K], recorded by the
    forward) holds w_vsA / w_vsB vertex-SDF candidates of A's / B's vertices
    and w_ee edge-edge witnesses: each window candidate is evaluated again
    (its QP from the distance pass's solution, its SDF queries) and swept in
    reverse; the distance pass (the QP of every edge pair) and the row /
    column LSE terms are recomputed, and the LSE terms swept in reverse.  The
    QP adjoints of the nearest-neighbour phase (edge pairs whose row or column
    softmax weight exceeds e^-28) are not counted: a lower bound."""
    vs_a = sdf_cost(kB, fB, True, True) + _VS
    vs_b = sdf_cost(kA, fA, True, False) + _VS
    ee = (_QP + _WITNESS + _INDICATORS + _NN_LSE
          + sdf_cost(kB, fB, False, True) + sdf_cost(kA, fA, True, False)
          + sdf_cost(kA, fA, False, False) + sdf_cost(kB, fB, True, True))
    visited = w_vsA * vs_a + w_vsB * vs_b + w_ee * ee
    nn = eA * eB * _NN_LSE
    return visited + _reverse(visited) + eA * eB * (_QP + _NN_LSE) + _reverse(nn)


def adjoint_batch_ops(types, nv, ne, nf, pairs_a, pairs_b, body_geom, w_vsA, w_vsB, w_ee) -> np.ndarray:
    """adjoint_pair_ops summed over kept pairs (per-pair window counts given)."""
    ga = body_geom[pairs_a]
    gb = body_geom[pairs_b]
    tot = np.zeros(3, dtype=np.int64)
    keys, inv = np.unique(np.stack([ga, gb]), axis=1, return_inverse=True)
    inv = inv.reshape(-1)
    cnt = np.bincount(inv, minlength=keys.shape[1])
    sa = np.bincount(inv, weights=w_vsA, minlength=keys.shape[1]).astype(np.int64)
    sb = np.bincount(inv, weights=w_vsB, minlength=keys.shape[1]).astype(np.int64)
    se = np.bincount(inv, weights=w_ee, minlength=keys.shape[1]).astype(np.int64)
    for j, (x, y) in enumerate(keys.T):
        # linear in the window counts and in the pair count
        base = adjoint_pair_ops(types[x], nv[x], ne[x], nf[x], types[y], nv[y], ne[y], nf[y], 0, 0, 0)
        per = adjoint_pair_ops(types[x], nv[x], ne[x], nf[x], types[y], nv[y], ne[y], nf[y], 1, 0, 0) - base
        per_b = adjoint_pair_ops(types[x], nv[x], ne[x], nf[x], types[y], nv[y], ne[y], nf[y], 0, 1, 0) - base
        per_e = adjoint_pair_ops(types[x], nv[x], ne[x], nf[x], types[y], nv[y], ne[y], nf[y], 0, 0, 1) - base
        tot += cnt[j] * base + sa[j] * per + sb[j] * per_b + se[j] * per_e
    return tot


# MI355X (gfx950): 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz
VALU_SLOTS_PER_S = 256 * 4 * 16 * 2.4e9      # full-rate lane operations per second
TRANS_SLOT_COST = 4                            # transcendental ops issue at a quarter rate


def roofline(ops: np.ndarray, seconds: float) -> dict:
    """ALU roofline: achieved flop rate vs the peak for this instruction mix."""
    fma, alu, trans = (float(x) for x in ops)
    flops = 2 * fma + alu + trans
    slots = fma + alu + TRANS_SLOT_COST * trans
    t_roof = slots / VALU_SLOTS_PER_S
    peak = flops / t_roof
    achieved = flops / seconds
    return dict(flops=flops, slots=slots, t_roof_s=t_roof, peak_flops=peak, achieved_flops=achieved,
                frac=achieved / peak)
