"""Plant plausible mistakes in the oracle (on the CPU) and check that the pins
catch every one of them.

Each mutation rewrites one line of one oracle function (source-level, in
memory) and monkeypatches the mutant in; at least one of the listed pins must
then fail.  This is what makes the pins evidence: a dropped term, a wrong sign,
a swapped index or a transposed operand in the oracle does not go unnoticed.
"""
import inspect
import textwrap

import pytest

from oracle import cm_oracle as O
from tests import oracle_pins as P

# the activity products of the two E-E witnesses, as the oracle writes them
_ACT = ('logG1 = qp["log_con"] + log_pen1 + log_nn1 + log_cl\n'
        '    logG2 = qp["log_con"] + log_pen2 + log_nn2 + log_cl')

# (oracle function, original text, mutated text, pins expected to catch it)
MUTATIONS = [
    ("ee_qp", "au1 = (-c1 * Q22 + Q12 * c2) / det", "au1 = (c1 * Q22 - Q12 * c2) / det",
     [P.pin_qp_hard_limit_segments, P.pin_qp_regularised_limit]),                      # text's sign slip
    ("ee_qp", "x_a = clip_s(-(Q12 + c2) / Q22, 0.0, 1.0, tau)", "x_a = clip_s(-(Q12 - c2) / Q22, 0.0, 1.0, tau)",
     [P.pin_qp_hard_limit_segments, P.pin_qp_regularised_limit]),                      # text's edge minimiser
    ("ee_qp", "costs = J(cand1, cand2)",
     "costs = J(cand1, cand2) + torch.stack([zero, zero, zero, c1 * (x_b - x_d)], dim=-1)",
     [P.pin_qp_hard_limit_segments, P.pin_qp_regularised_limit, P.pin_qp_edge_swap_symmetry]),  # listing cost bug
    ("ee_qp", "Q11 = _dot(t1, t1) + lam", "Q11 = _dot(t1, t1)",
     [P.pin_qp_regularised_limit, P.pin_qp_edge_swap_symmetry]),                      # dropped regulariser
    ("ee_qp", "con = within_s(au1, 0.0, 1.0, tau) * within_s(au2, 0.0, 1.0, tau)",
     "con = within_s(au1, 0.0, 1.0, tau) * within_s(au1, 0.0, 1.0, tau)",
     [P.pin_qp_hard_limit_segments, P.pin_qp_edge_swap_symmetry]),                    # wrong index
    ("ee_qp", "pi = argmin_s(costs, tau, dim=-1)", "pi = argmin_s(-costs, tau, dim=-1)",
     [P.pin_qp_hard_limit_segments, P.pin_qp_regularised_limit]),                      # soft argmax
    ("ee_sign", "sign_s(_dot(gA_e1, -nbar), tau)", "sign_s(_dot(gA_e1, nbar), tau)",
     [P.pin_crossing_edges_sign]),                                                     # literal "vice versa"
    ("ee_sign", "return sign_s(_dot(gB_e2, nbar), tau)", "return sign_s(_dot(gB_e2, -nbar), tau)",
     [P.pin_crossing_edges_sign]),
    ("nn_log_indicators", "torch.log_softmax(-dbar / tau, dim=1), torch.log_softmax(-dbar / tau, dim=0)",
     "torch.log_softmax(-dbar / tau, dim=0), torch.log_softmax(-dbar / tau, dim=1)",
     [P.pin_nn_rows_columns]),                                                         # transposed nn
    ("vs_normal", "torch.sqrt(tau + _dot(g, g))", "torch.sqrt(_dot(g, g))",
     [P.pin_vs_normal_sphere]),                                                        # dropped tau
    ("pair_candidates", "vs_nu = torch.cat([-vs_normal(gB_v, tau), vs_normal(gA_v, tau)])",
     "vs_nu = torch.cat([vs_normal(gB_v, tau), vs_normal(gA_v, tau)])",
     [P.pin_vs_normal_sphere, P.pin_pair_swap_antisymmetry]),                          # V-S normal sign
    ("pair_candidates", "vs_logw = log_sigmoid(-vs_d / tau)", "vs_logw = log_sigmoid(vs_d / tau)",
     [P.pin_vs_weights_point_in_polytope]),                                            # inverted pen test
    ("pair_candidates", "log_pen1 = log_sigmoid(-phiB_e1 / tau)", "log_pen1 = log_sigmoid(-phiA_e2 / tau)",
     [P.pin_pair_swap_antisymmetry]),                                                  # wrong SDF for pen
    # symmetric mistakes in the activity product (both witnesses alike)
    ("pair_candidates", _ACT, _ACT.replace('qp["log_con"] + ', ""),
     [P.pin_ee_activity_hard_limit]),                                                  # dropped con
    ("pair_candidates", _ACT, _ACT.replace("log_pen1 + ", "").replace("log_pen2 + ", ""),
     [P.pin_ee_activity_hard_limit]),                                                  # dropped pen
    ("pair_candidates", _ACT, _ACT.replace(" + log_cl", ""),
     [P.pin_ee_activity_hard_limit]),                                                  # dropped cl
    ("pair_candidates", _ACT, _ACT.replace("log_nn1 + ", "").replace("log_nn2 + ", ""),
     [P.pin_ee_activity_hard_limit]),                                                  # dropped nn
    ("pair_candidates", _ACT, _ACT.replace("log_nn1", "@").replace("log_nn2", "log_nn1").replace("@", "log_nn2"),
     [P.pin_ee_activity_hard_limit]),                                                  # nn rows <-> columns
    ("log_within_s", "return log_sigmoid((x - lo) / tau) + log_sigmoid((hi - x) / tau)",
     "return log_sigmoid((x - lo) / tau)", [P.pin_ee_activity_hard_limit]),           # upper side dropped
    ("log_within_s", "return log_sigmoid((x - lo) / tau) + log_sigmoid((hi - x) / tau)",
     "return log_sigmoid((hi - x) / tau)", [P.pin_ee_activity_hard_limit]),           # lower side dropped
    ("manifold", "torch.softmax(-torch.abs(top[:, None] - s[None, :]) / tau, dim=1)",
     "torch.softmax(-(top[:, None] - s[None, :]) / tau, dim=1)",
     [P.pin_manifold_properties]),                                                     # SoftSort without |.|
    ("manifold", "top = torch.topk(s, k, sorted=True).values", "top = torch.topk(s, k, largest=False).values",
     [P.pin_manifold_properties]),                                                     # bottom-K
    ("manifold", "out[key] = torch.cat([out[key], out[key].new_zeros(pad)])",
     "out[key] = torch.cat([out[key], out[key].new_ones(pad)])",
     [P.pin_simplification_flags]),                                                    # empty rows not empty
    ("pair_candidates", "vs_p, vs_nu, vs_d, vs_logw = vs_p[:nA], vs_nu[:nA], vs_d[:nA], vs_logw[:nA]",
     "vs_p, vs_nu, vs_d, vs_logw = vs_p[-nA:], vs_nu[-nA:], vs_d[-nA:], vs_logw[-nA:]",
     [P.pin_simplification_flags]),                                                    # one-sided keeps B's side
    ("ee_qp_hard", "torch.clamp(-(Q12 + c2) / Q22, 0.0, 1.0)", "torch.clamp(-(Q12 - c2) / Q22, 0.0, 1.0)",
     [P.pin_qp_no_smoothing]),                                                         # edge minimiser sign
    ("ee_qp_hard", "best = torch.argmin(costs, dim=-1, keepdim=True)", "best = torch.argmax(costs, dim=-1, keepdim=True)",
     [P.pin_qp_no_smoothing]),                                                         # worst box edge
    ("preselect", "meA = 0.5 * (mA[eA[:, 0]] + mA[eA[:, 1]])", "meA = torch.maximum(mA[eA[:, 0]], mA[eA[:, 1]])",
     [P.pin_preselect_against_sphere]),                                                # edge metric not the mean
    ("preselect", "GvA = soft_topk(-mA, min(KV, vA.shape[0]), tau)", "GvA = soft_topk(mA, min(KV, vA.shape[0]), tau)",
     [P.pin_preselect_against_sphere]),                                                # shallowest selected
    ("soft_topk", "top = torch.topk(x, K, sorted=True).values", "top = torch.topk(x, K, sorted=False).values",
     [P.pin_soft_topk]),                                                               # rows out of order
    ("quat_to_R", "[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)]",
     "[1 - 2 * (y * y + z * z), 2 * (x * y + w * z), 2 * (x * z + w * y)]",
     [P.pin_quaternion_rotation]),                                                     # sign in R
    ("pose_Rt", "return R + W @ R, t + xi[:3] + W @ t", "return R + R @ W, t + R @ xi[:3]",
     [P.pin_gradient_joint_motion_identities]),                                        # body-frame twist
    ("sdf_local", "return nrm - r, y / nrm[..., None]", "return nrm - r, -y / nrm[..., None]",
     [P.pin_sdf_gradients_fd]),                                                        # capsule normal sign
    ("sdf_local", "zc = torch.minimum(torch.maximum(x[..., 2], -h), h)", "zc = torch.maximum(x[..., 2], -h)",
     [P.pin_analytic_sdf_brute_force]),                                                # capsule clamp
    ("sdf_local", "phi = torch.where(outside, n_out, torch.zeros_like(s)) + torch.clamp(qmax, max=0.0) - rho",
     "phi = torch.where(outside, n_out, torch.zeros_like(s)) + torch.clamp(qmax, max=0.0) + rho",
     [P.pin_analytic_sdf_brute_force]),                                                # rounding sign
    ("planes", "o = (n * v0).sum(-1)", "o = (n * (v0 - v1)).sum(-1)",
     [P.pin_hull_counts, P.pin_polytope_inside_delaunay]),                             # plane offset
    ("hull_topology", "if np.dot(n, eq[:3]) < 0:", "if np.dot(n, eq[:3]) > 0:",
     [P.pin_hull_counts, P.pin_polytope_inside_delaunay]),                             # inward normals
    ("broadphase", "keep = d2 <= r * r", "keep = d2 <= r",
     [P.pin_broadphase_f32]),                                                          # missing square
    ("sq_union_sdf", "phi_i = r * (1.0 - q)", "phi_i = (1.0 - q) / r",
     [P.pin_sq_axis_distance]),                                                        # printed division by |x|
    ("sq_union_sdf", "q = f ** (-e1 / 2.0)", "q = f ** (-e2 / 2.0)",
     [P.pin_sq_axis_distance]),                                                        # wrong exponent
    ("sq_inside_outside", "torch.where(upos, us ** (e2 / e1), torch.zeros_like(u)) + C",
     "torch.where(upos, us ** (e1 / e2), torch.zeros_like(u)) + C",
     [P.pin_sq_axis_distance, P.pin_sq_surface_and_mesh]),                             # inverted ratio
    ("sq_union_sdf", "phi = -lse_t(-phi_i, tau, dim=-1)", "phi = lse_t(phi_i, tau, dim=-1)",
     [P.pin_sq_union_bounds]),                                                         # smooth max
    ("sq_inside_outside", "dC = 2.0 / e1 * _spow(s[..., 2], 2.0 / e1 - 1.0)",
     "dC = 2.0 / e1 * _spow(s[..., 2], 2.0 / e2 - 1.0)",
     [P.pin_sq_gradients_fd]),                                                         # gradient exponent
    ("sq_points", "ax[i, 0] * _spow(ce, e1[i]) * _spow(co, e2[i])", "ax[i, 0] * _spow(ce, e2[i]) * _spow(co, e1[i])",
     [P.pin_sq_surface_and_mesh]),                                                     # swapped exponents
    ("sq_union_mesh", "inside = [(j != i) and bool(f[j] < 1.0) for j in range(M)]",
     "inside = [(j != i) and bool(f[j] > 1.0) for j in range(M)]",
     [P.pin_sq_surface_and_mesh]),                                                     # pruned the outside
    ("sphere_trace", "x = x - phi[..., None] * n", "x = x + phi[..., None] * n",
     [P.pin_sphere_trace_metric_one_step, P.pin_sphere_trace_polytope_converges]),      # steps away
    ("pair_candidates", "e1 = sphere_trace(GA, RA, tA, e1, tau, planesA, refine)",
     "e1 = sphere_trace(GB, RB, tB, e1, tau, planesB, refine)",
     [P.pin_refined_witnesses_on_own_surfaces]),                                       # traced on the wrong body
    ("opc_sdf", "grad = (w[..., None] * (n + dlb * (h - phi[..., None])[..., None])).sum(-2)",
     "grad = (w[..., None] * n).sum(-2)",
     [P.pin_opc_gradient_fd]),                                                         # dropped weight derivative
    ("opc_sdf", "lb = -(d * d).sum(-1) / (2.0 * sg * sg)", "lb = -(d * d).sum(-1) / (sg * sg)",
     [P.pin_opc_gradient_fd]),                                                         # kernel width
    ("opc_sdf", "h = (d * n).sum(-1)", "h = -(d * n).sum(-1)",
     [P.pin_opc_single_point_and_plane]),                                              # inward normals
    ("opc_knn_edges", "order = sorted(range(len(P)), key=lambda j: (d2[j], j))[:min(k, len(P) - 1)]",
     "order = sorted(range(len(P)), key=lambda j: (d2[j], j))[:min(k + 1, len(P) - 1)]",
     [P.pin_opc_knn_edges]),                                                           # k + 1 neighbours
]


def _mutant(fn_name, old, new):
    owner = O.OGeom if fn_name == "planes" else O
    src = textwrap.dedent(inspect.getsource(getattr(owner, fn_name)))
    assert src.count(old) == 1, (fn_name, old)
    ns = {}
    exec(compile(src.replace(old, new), f"<mutant {fn_name}>", "exec"), O.__dict__, ns)
    return owner, ns[fn_name]


@pytest.mark.parametrize("mut", MUTATIONS, ids=[f"{m[0]}:{i}" for i, m in enumerate(MUTATIONS)])
def test_mutation_is_caught(mut, monkeypatch):
    fn_name, old, new, pins = mut
    owner, fn = _mutant(fn_name, old, new)
    monkeypatch.setattr(owner, fn_name, fn)
    caught = []
    for pin in pins:
        try:
            pin()
        except (AssertionError, RuntimeError, ValueError, IndexError):
            caught.append(pin.__name__)
    assert caught, f"mutation of {fn_name} ({new!r}) was not caught by {[p.__name__ for p in pins]}"
