"""The oracle's pins catch plausible mistakes.

Each mutant is a copy of oracle/etac_oracle.c with one planted mistake (a
flipped inequality, a dropped term, a wrong sign or index, a transposed
concatenation).  It is compiled on the CPU and loaded in place of the oracle,
and the pin tests are run against it: at least one pin must fail.  The real
oracle is restored afterwards."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

import oracle
from tests import test_oracle_adjoint as TA
from tests import test_oracle_contact as TC
from tests import test_oracle_hand as TH
from tests import test_oracle_mesh as TM
from tests import test_oracle_propagate as TP
from tests import test_oracle_regress as TR

SRC = oracle.SRC

# (name, original text, mutated text)
MUTANTS = [
    ("surface nodes active", "if (!(s < r * r)) return h;\n        h.inside = 1;\n        if (s == 0.0) {\n            h.degenerate = 1;\n            h.depth = r;\n            for (int a = 0; a < 3; ++a) h.u[a] = -r * nrm[a];\n            return h;\n        }\n        double l = sqrt(s);\n        h.depth = r - l;\n        double sc = h.depth / l;\n        h.u[0]",
     "if (!(s <= r * r)) return h;\n        h.inside = 1;\n        if (s == 0.0) {\n            h.degenerate = 1;\n            h.depth = r;\n            for (int a = 0; a < 3; ++a) h.u[a] = -r * nrm[a];\n            return h;\n        }\n        double l = sqrt(s);\n        h.depth = r - l;\n        double sc = h.depth / l;\n        h.u[0]"),
    ("box face tie to highest axis", "if (sl < best) { best = sl; cs = c; }\n        }\n        h.face = cs;",
     "if (sl <= best) { best = sl; cs = c; }\n        }\n        h.face = cs;"),
    ("capsule ignores clamp", "double v0 = q[0], v1 = q[1], v2 = q[2] - z;", "double v0 = q[0], v1 = q[1], v2 = q[2];"),
    ("shallowest object wins", "P->trans + 3 * eo, p, n);\n                if (h.inside && (best < 0 || h.depth > bh.depth))",
     "P->trans + 3 * eo, p, n);\n                if (h.inside && (best < 0 || h.depth < bh.depth))"),
    ("mesh contact: shallowest object wins",
     "continue;\n                }\n                if (h.inside && (best < 0 || h.depth > bh.depth)) { best = o; bh = h; }",
     "continue;\n                }\n                if (h.inside && (best < 0 || h.depth < bh.depth)) { best = o; bh = h; }"),
    ("decay uses squared distance", "return exp(-alpha * d);", "return exp(-alpha * d * d);"),
    ("decay sums the passive node", "for (int a = 0; a < 3; ++a) acc[a] += w * uhat[(size_t)a * E * N + ej];",
     "for (int a = 0; a < 3; ++a) acc[a] += w * uhat[(size_t)a * E * N + (size_t)e * N + i];"),
    ("network input p + o", "x[a] = P->pos[(size_t)a * N + i] - P->origin[3 * k + a];",
     "x[a] = P->pos[(size_t)a * N + i] + P->origin[3 * k + a];"),
    ("concat [g'; f]", "for (int c = 0; c < NF; ++c) acc += W->W4[o * 2 * NF + c] * f[c];\n        for (int c = 0; c < NF; ++c) acc += W->W4[o * 2 * NF + NF + c] * gp[c];",
     "for (int c = 0; c < NF; ++c) acc += W->W4[o * 2 * NF + c] * gp[c];\n        for (int c = 0; c < NF; ++c) acc += W->W4[o * 2 * NF + NF + c] * f[c];"),
    ("min-pool", "if (S->f[(size_t)li * NF + c] > best) { best = S->f[(size_t)li * NF + c]; am = li; }",
     "if (S->f[(size_t)li * NF + c] < best) { best = S->f[(size_t)li * NF + c]; am = li; }"),
    ("residual on active nodes", "int i = S->pas[t];\n            int li = i - P->offset[k];\n            phi_decode",
     "int i = S->pas[t] == P->offset[k] ? S->act[0] : S->pas[t];\n            int li = i - P->offset[k];\n            phi_decode"),
    ("alpha gradient sign", "da += -d * w * dot;", "da += d * w * dot;"),
    ("sphere pose gradient sign", "for (int a = 0; a < 3; ++a) gt[a] += -(phi * g[a] + twophip * gd * d[a]);",
     "for (int a = 0; a < 3; ++a) gt[a] += (phi * g[a] + twophip * gd * d[a]);"),
    ("box rotation gradient term", "gR[a * 3 + cs] += coef * g[a] - grc * d[a];", "gR[a * 3 + cs] += coef * g[a] + grc * d[a];"),
    ("capsule drops the axial projection", "if (!clamped) av[2] = twophip * gRv * v[2];", ""),
    ("max-pool routes to node 0", "S->df[(size_t)S->argmax[c] * NF + c] += dg[c];", "S->df[(size_t)0 * NF + c] += dg[c];"),
    ("decoder gradient misses W4 g' part", "dW->W4[o * 2 * NF + NF + c] += dh4[o] * S->gp[c];", "dW->W4[o * 2 * NF + NF + c] += dh4[o] * S->g[c];"),
    ("encoder gate uses h1 instead of pre1", "dpre1[c] = pre1[c] > 0.0 ? acc : 0.0;", "dpre1[c] = acc;"),
    ("mesh sign from the face normal only", "if (!(dot3(w, m->pn + bf * 21 + bfeat * 3) < 0.0)) return h;",
     "if (!(dot3(w, m->pn + bf * 21) < 0.0)) return h;"),
    ("mesh edge ab parameter", "double v = d1 / (d1 - d3);", "double v = d3 / (d1 - d3);"),
    ("mesh u_hat points inward", "double v[3] = {bcp[0] - q[0], bcp[1] - q[1], bcp[2] - q[2]};",
     "double v[3] = {q[0] - bcp[0], q[1] - bcp[1], q[2] - bcp[2]};"),
    ("mesh adjoint drops the frame term", "gR[a * 3 + b] += g[a] * w[b] + d[a] * h[b];", "gR[a * 3 + b] += g[a] * w[b];"),
    ("mesh edge Jacobian as a vertex", "J[i * 3 + j] = e[i] * e[j] / ee - (i == j ? 1.0 : 0.0);",
     "J[i * 3 + j] = -(i == j ? 1.0 : 0.0);"),
    ("u_hat gradient from passive input", "if (cobj[ei] >= 0) { /* only active nodes carry u_hat into the input */",
     "if (cobj[ei] < 0) { /* only active nodes carry u_hat into the input */"),
    ("hand: relative rotation without the transpose",
     "Rr[a * 3 + c] = sum3(Rl[0 * 3 + a] * Rw[0 * 3 + c], Rl[1 * 3 + a] * Rw[1 * 3 + c],\n                                 Rl[2 * 3 + a] * Rw[2 * 3 + c]);",
     "Rr[a * 3 + c] = sum3(Rl[a * 3 + 0] * Rw[0 * 3 + c], Rl[a * 3 + 1] * Rw[1 * 3 + c],\n                                 Rl[a * 3 + 2] * Rw[2 * 3 + c]);"),
    ("hand: translation not taken relative to the link", "double d[3] = {tw[0] - tl[0], tw[1] - tl[1], tw[2] - tl[2]};",
     "double d[3] = {tw[0], tw[1], tw[2]};"),
    ("hand: link primitive offset ignored",
     "C->tw[s][a] = sum3(Rj[a * 3 + 0] * Ct[0], Rj[a * 3 + 1] * Ct[1], Rj[a * 3 + 2] * Ct[2]) + tj[a];",
     "C->tw[s][a] = tj[a];"),
    ("hand: frame-link translation gradient sign", "gtl[a] -= gtw[a];", "gtl[a] += gtw[a];"),
    ("hand: frame-link rotation gradient drops the lever term", "gRl[a * 3 + b] += v + d[a] * gt[s][b];",
     "gRl[a * 3 + b] += v;"),
    ("hand: object gradient left in the link frame", "for (int i = 0; i < 9; ++i) go[i] += GRw[i];",
     "for (int i = 0; i < 9; ++i) go[i] += gR[s][i];"),
    ("hand: link primitive gradient drops its offset", "GRw[a * 3 + 2] * CR[b * 3 + 2] + gtw[a] * Ct[b];",
     "GRw[a * 3 + 2] * CR[b * 3 + 2];"),
    ("hand: reward counts self-contact", "if (C->id[s] < O) ++nt;", "++nt;"),
    ("hand: reward without the empty-contact penalty", "double ra = s > 0 ? (double)s / (double)P->N : -0.1;",
     "double ra = s > 0 ? (double)s / (double)P->N : 0.0;"),
    ("regressor: no residual connection", "h2[o] = relu(a) + h1[o];", "h2[o] = relu(a);"),
    ("regressor: attention weights not normalised", "g[c] = a / z;", "g[c] = a;"),
    ("regressor: relu instead of tanh in the attention", "t[o] = tanh(a);", "t[o] = relu(a);"),
    ("regressor: positions not relative to the origin", "x[a] = pos[(size_t)a * N + i] - origin[3 * k + a];",
     "x[a] = pos[(size_t)a * N + i];"),
    ("regressor: head without its hidden relu", "h[o] = relu(a);\n                }\n                double *yo",
     "h[o] = a;\n                }\n                double *yo"),
]


def _pins():
    """Quick pins, each a zero-argument callable raising on failure."""
    P = pytest.mark.parametrize
    return [
        lambda o: TC.test_sphere_worked_example_node_below_centre(o),
        lambda o: TC.test_sphere_active_set_exact_rational(o, 0),
        lambda o: [TC.test_penetration_vs_brute_force_surface_sampling(o, t) for t in (0, 1, 2)],
        lambda o: TC.test_deepest_object_wins_and_ties_to_lowest_index(o),
        lambda o: TC.test_box_face_tie_goes_to_lowest_axis_and_zero_is_positive(o),
        lambda o: TC.test_surface_nodes_are_passive(o),
        lambda o: TP.test_decay_equals_explicit_omega_matmul(o, 0),
        lambda o: TP.test_golden_two_node_hand_example(o),
        lambda o: TP.test_full_is_sum_of_ablations_on_passive_nodes(o),
        lambda o: [TP.test_forward_vs_independent_torch_float64(o, m) for m in (0, 1, 2)],
        lambda o: TA.test_contact_adjoint_vs_torch_autograd(o),
        lambda o: [TA.test_propagation_adjoint_vs_torch_autograd(o, m) for m in (0, 1, 2)],
        lambda o: TA.test_raw_rotation_entries_vs_fd(o),
        lambda o: TM.test_closest_point_vs_independent_and_sampling(o),
        lambda o: TM.test_convex_hull_inside_and_depth_vs_qhull_planes(o),
        lambda o: TM.test_triangulated_cube_matches_box_primitive(o),
        lambda o: TM.test_deepest_object_wins_across_primitives_and_meshes(o),
        lambda o: [TM.test_mesh_pose_adjoint_vs_central_differences(o, m) for m in (0, "L")],
        lambda o: TM.test_mesh_adjoint_with_a_primitive_and_raw_rotation_entries(o),
        lambda o: TH.test_identity_links_reduce_to_the_plain_step(o),
        lambda o: TH.test_link_frame_contact_equals_world_frame_contact(o),
        lambda o: TH.test_self_contact_sphere_closed_form(o),
        lambda o: TH.test_rigid_motion_of_everything_changes_nothing(o),
        lambda o: TH.test_adjoint_translation_and_rotation_sums_vanish(o),
        lambda o: TH.test_contact_reward_worked_example(o),
        lambda o: [TH.test_hand_pose_adjoint_vs_central_differences(o, m) for m in (1, 0)],
        lambda o: TR.test_closed_form_softmax_weighted_mean(o),
        lambda o: TR.test_single_node_and_uniform_attention(o),
        lambda o: TR.test_node_order_duplication_and_score_shift_change_nothing(o),
        lambda o: TR.test_residual_connection(o),
    ]


def _caught(lib_path):
    saved = oracle._lib
    oracle._lib = C.CDLL(lib_path)
    try:
        for pin in _pins():
            try:
                pin(oracle)
            except (AssertionError, ValueError, RuntimeError, IndexError):
                return True
        return False
    finally:
        oracle._lib = saved


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(tmp_path, oracle_lib, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutant anchor not unique: {name}"
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                           "-fno-fast-math", "-w", str(path), "-o", str(lib), "-lm"])
    assert _caught(str(lib)), f"no pin caught the planted mistake: {name}"


def test_unmutated_oracle_passes_the_same_pins(oracle_lib):
    assert not _caught(oracle.LIB)
