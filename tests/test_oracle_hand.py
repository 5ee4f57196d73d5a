"""Pins of the oracle's articulated-hand step (link frames, self-contact,
contact reward) against what geometry and the mathematics fix:

- with every link at the identity pose and no self-contact pairs the hand
  step is the plain step, bit for bit (forward and object adjoint);
- contact evaluated in each link's frame equals contact evaluated in the
  world frame by the plain contact pass on world-frame node positions, with
  the other links' primitives as objects;
- a node inside another link's sphere gets the closed-form displacement;
- a rigid motion of the whole scene leaves every output unchanged, and the
  adjoint's translation and rotation sums over all bodies vanish;
- the contact reward of a worked example (a box pressed on the flat palm
  grid: the touched nodes are counted from the grid) and the paper's
  piecewise rule for n_a = 0 (Sec. IV-B, contact reward);
- the pose adjoint against central differences, for object poses, for the
  frame link of a patch and for a link whose primitive touches another
  link's patch."""
from dataclasses import replace

import numpy as np
import pytest

import oracle
import scenes
from scenes import articulated as art

O_MAX = 2


def _model(mesh, mode=scenes.MODE_FULL, seed=3):
    return scenes.draw_model(np.random.default_rng([seed, 5]), mesh.pitch, mode)


def _identity_hand(K):
    """K links, one patch each, no primitives, no self-contact pairs."""
    return art.Hand(K, np.full(K, -1, np.int32), np.arange(K, dtype=np.int32), np.zeros(K, np.uint32),
                    np.full(K, art.NONE, np.int32), np.zeros((K, 4), np.float32),
                    np.tile(np.eye(3, dtype=np.float32).ravel(), (K, 1)), np.zeros((K, 3), np.float32),
                    np.zeros((K, 3)), np.tile(np.eye(3), (K, 1, 1)))


def _rodrigues(w):
    return oracle.expm_so3(np.asarray(w, np.float64))


def test_identity_links_reduce_to_the_plain_step(oracle_lib):
    mesh, scene, model = scenes.config2(n_envs=12)
    h = _identity_hand(mesh.n_patches)
    lk = art.identity_links(h, scene.n_envs)
    a = oracle.hand_forward(mesh, h, scene, lk, model)
    b = oracle.forward(mesh, scene, model)
    for key in ("u", "uhat", "contact_obj", "n_active"):
        assert np.array_equal(a[key], b[key]), key
    assert np.array_equal(a["n_touch"], a["n_active"])
    w = np.random.default_rng(2).standard_normal(b["u"].shape)
    ga = oracle.hand_backward(mesh, h, scene, lk, model, w)
    gb = oracle.backward(mesh, scene, model, w)
    for key in ("grad_alpha", "grad_phi"):
        assert np.array_equal(ga[key], gb[key]), key
    # pose partials are summed per patch first here: equal up to that order
    for key in ("grad_rot", "grad_trans"):
        assert np.allclose(ga[key], gb[key], rtol=1e-12, atol=1e-12 * np.abs(gb[key]).max()), key
    # moving a link's frame by d moves its patch relative to every object by -d
    sum_obj = np.zeros_like(gb["grad_trans"][:, 0])
    for e in range(scene.n_envs):
        sum_obj[e] = gb["grad_trans"][e, : scene.n_obj[e]].sum(axis=0)
    assert np.allclose(ga["grad_link_trans"].sum(axis=1), -sum_obj, rtol=1e-9, atol=1e-9)


def _world_patch_mesh(mesh, k, R, t):
    a, b = int(mesh.patch_offset[k]), int(mesh.patch_offset[k + 1])
    p = mesh.pos[:, a:b].astype(np.float64)
    n = mesh.nrm[:, a:b].astype(np.float64)
    return scenes.Mesh(np.array([0, b - a], np.int32), R @ p + t[:, None], R @ n, np.zeros((1, 3)),
                       np.ones(1), [])


def _orthonormal_links(links):
    """FP64 link poses with exactly orthonormal rotations (polar factor of
    the FP32 matrices), so that link-frame and world-frame evaluations agree
    to FP64 rounding."""
    R = links.rot.reshape(*links.rot.shape[:2], 3, 3).astype(np.float64)
    U, _, Vt = np.linalg.svd(R)
    return art.Links((U @ Vt).reshape(links.rot.shape), links.trans.astype(np.float64))


def test_link_frame_contact_equals_world_frame_contact(oracle_lib):
    h, mesh = art.hand()
    scene, links = art.grasp_scene(h, mesh, 10, seed=4)
    links = _orthonormal_links(links)
    model = _model(mesh)
    out = oracle.hand_forward(mesh, h, scene, links, model, rel32=False)
    O = scene.max_obj
    n_self = 0
    for e in range(scene.n_envs):
        for k in range(mesh.n_patches):
            l = int(h.patch_link[k])
            Rl = links.rot[e, l].reshape(3, 3).astype(np.float64)
            tl = links.trans[e, l].astype(np.float64)
            wm = _world_patch_mesh(mesh, k, Rl, tl)
            # world scene: the env's objects, then the primitives of the links in collide[l]
            ids, typ, shp, rot, tr = [], [], [], [], []
            for o in range(scene.n_obj[e]):
                ids.append(o); typ.append(scene.type[e, o]); shp.append(scene.shape[e, o])
                rot.append(scene.rot[e, o].astype(np.float64)); tr.append(scene.trans[e, o].astype(np.float64))
            for j in range(h.n_links):
                if j == l or not (int(h.collide[l]) >> j) & 1:
                    continue
                Rj = links.rot[e, j].reshape(3, 3).astype(np.float64)
                tj = links.trans[e, j].astype(np.float64)
                CR = h.prim_rot[j].reshape(3, 3).astype(np.float64)
                Ct = h.prim_trans[j].astype(np.float64)
                ids.append(O + j); typ.append(h.prim_type[j]); shp.append(h.prim_shape[j])
                rot.append((Rj @ CR).ravel()); tr.append(Rj @ Ct + tj)
            n = len(ids)
            ws = scenes.Scene(np.array([n], np.int32), np.array([typ], np.int32), np.array([shp], np.float64),
                              np.array([rot], np.float64), np.array([tr], np.float64))
            cw, uw, _ = oracle.contact(wm, ws)
            a, b = int(mesh.patch_offset[k]), int(mesh.patch_offset[k + 1])
            got = out["contact_obj"][e, a:b]
            exp = np.where(cw[0] >= 0, np.array(ids + [-1])[cw[0]], -1)
            assert np.array_equal(got, exp), (e, k)
            n_self += int((got >= O).sum())
            u_world = Rl @ out["uhat"][:, e, a:b]
            assert np.allclose(u_world, uw[:, 0], rtol=0, atol=1e-9), (e, k)
    assert n_self > 0   # the workload has self-contact


def test_self_contact_sphere_closed_form(oracle_lib):
    # link 0 carries a 5x5 flat patch (1 mm pitch) at z = 0 of its frame; link 1
    # is a sphere of radius 2.9 centred 2 mm above the patch centre (link-0
    # frame); link 0 is rotated and shifted in the world
    pos, nrm = art._flat_patch(5, 5, 1.0, 0.0)
    mesh = scenes.Mesh(np.array([0, 25], np.int32), pos.astype(np.float32), nrm.astype(np.float32),
                       np.zeros((1, 3), np.float32), np.ones(1), [])
    h = art.Hand(2, np.array([-1, -1], np.int32), np.array([0], np.int32), np.array([0b10, 0b01], np.uint32),
                 np.array([art.NONE, scenes.SPHERE], np.int32), np.array([[0, 0, 0, 0], [2.9, 0, 0, 0]], np.float32),
                 np.tile(np.eye(3, dtype=np.float32).ravel(), (2, 1)), np.zeros((2, 3), np.float32),
                 np.zeros((2, 3)), np.tile(np.eye(3), (2, 1, 1)))
    R0 = _rodrigues([0.3, -0.5, 0.2])
    t0 = np.array([10.0, -4.0, 7.0])
    c_local = np.array([0.0, 0.0, 2.0])
    lk = art.Links(np.array([[R0.ravel(), np.eye(3).ravel()]]), np.array([[t0, R0 @ c_local + t0]]))
    sc = scenes._empty_scene(1, 1)
    out = oracle.hand_forward(mesh, h, sc, lk, _model(mesh, scenes.MODE_DECAY_ONLY), rel32=False)
    p = pos.T
    d = p - c_local
    dist = np.linalg.norm(d, axis=1)
    r = float(np.float32(2.9))
    inside = dist < r
    assert inside.sum() == 9 + 4     # x^2 + y^2 < r^2 - 4 = 4.41: |x|, |y| <= 1 and (+-2, 0), (0, +-2)
    assert np.array_equal(out["contact_obj"][0], np.where(inside, 1 + 1, -1))   # id O + j with O = 1, j = 1
    exp_u = ((r - dist) / dist)[:, None] * d
    exp_u[~inside] = 0.0
    assert np.allclose(out["uhat"][:, 0].T, exp_u, rtol=0, atol=1e-12)
    assert out["n_touch"][0, 0] == 0 and out["n_active"][0, 0] == 13 and out["n_a"][0] == 0


def _random_motion(scene, links, seed):
    rng = np.random.default_rng(seed)
    G = scenes.random_rotation(rng)
    g = rng.uniform(-80, 80, size=3)
    S = scene.copy()
    S.rot = np.einsum("ab,eobc->eoac", G, scene.rot.reshape(*scene.rot.shape[:2], 3, 3).astype(np.float64)).reshape(
        scene.rot.shape)
    S.trans = scene.trans.astype(np.float64) @ G.T + g
    lk = art.Links(np.einsum("ab,elbc->elac", G, links.rot.reshape(*links.rot.shape[:2], 3, 3).astype(
        np.float64)).reshape(links.rot.shape), links.trans.astype(np.float64) @ G.T + g)
    return S, lk


def test_rigid_motion_of_everything_changes_nothing(oracle_lib):
    h, mesh = art.hand()
    scene, links = art.grasp_scene(h, mesh, 8, seed=5)
    model = _model(mesh)
    a = oracle.hand_forward(mesh, h, scene, links, model, rel32=False)
    S, lk = _random_motion(scene, links, 9)
    b = oracle.hand_forward(mesh, h, S, lk, model, rel32=False)
    assert np.array_equal(a["contact_obj"], b["contact_obj"])
    assert np.allclose(a["u"], b["u"], rtol=0, atol=1e-9)
    assert np.array_equal(a["n_a"], b["n_a"]) and np.array_equal(a["link_mask"], b["link_mask"])


def test_adjoint_translation_and_rotation_sums_vanish(oracle_lib):
    # L is invariant under moving every body (objects and links) together, so
    # sum_b dL/dt_b = 0 and sum_b (twist_b + t_b x dL/dt_b) = 0
    h, mesh = art.hand()
    scene, links = art.grasp_scene(h, mesh, 8, seed=6)
    model = _model(mesh)
    w = np.random.default_rng(1).standard_normal((3, scene.n_envs, mesh.n_nodes))
    g = oracle.hand_backward(mesh, h, scene, links, model, w, rel32=False)
    for e in range(scene.n_envs):
        bodies = [(scene.rot[e, o], scene.trans[e, o], g["grad_rot"][e, o], g["grad_trans"][e, o])
                  for o in range(scene.n_obj[e])]
        bodies += [(links.rot[e, l], links.trans[e, l], g["grad_link_rot"][e, l], g["grad_link_trans"][e, l])
                   for l in range(h.n_links)]
        st = sum(b[3] for b in bodies)
        sr = sum(oracle.twist_from_grad_rot(b[2], b[0]) + np.cross(b[1].astype(np.float64), b[3]) for b in bodies)
        scale = max(1.0, max(np.abs(b[3]).max() for b in bodies))
        assert np.abs(st).max() <= 1e-9 * scale, e
        assert np.abs(sr).max() <= 1e-7 * scale, e


def test_contact_reward_worked_example(oracle_lib):
    # a box of half extents (10, 5, 4) with centre 2 mm above the palm face
    # presses 2 mm into it: the palm grid (2.5 mm pitch, nodes at +-1.25,
    # +-3.75, ...) has 8 x 4 nodes with |x| < 10 and |y| < 5.  Fingers open
    # (identity joint angles) and far from the box.
    h, mesh = art.hand()
    R, t = art.forward_kinematics(h, np.zeros((h.n_links, 2)), np.eye(3), np.zeros(3))
    lk = art.Links(R.reshape(1, h.n_links, 9).astype(np.float32), t.reshape(1, h.n_links, 3).astype(np.float32))
    sc = scenes._empty_scene(1, O_MAX)
    sc.n_obj[0] = 1
    sc.type[0, 0] = scenes.BOX
    sc.shape[0, 0, :3] = (10.0, 5.0, 4.0)
    sc.trans[0, 0] = (0.0, 0.0, art.PALM_HALF[2] + 2.0)
    out = oracle.hand_forward(mesh, h, sc, lk, _model(mesh), omega_a=0.5)
    assert out["n_touch"][0, 0] == 32 and out["n_touch"][0, 1:].sum() == 0
    assert out["n_a"][0] == 32 and out["link_mask"][0] == 1
    assert out["r_contact"][0] == pytest.approx(1.0 / 16.0 + 0.5 * 32.0 / mesh.n_nodes, rel=1e-15)
    # no object: the -0.1 branch, no link touched
    sc.n_obj[0] = 0
    out = oracle.hand_forward(mesh, h, sc, lk, _model(mesh), omega_a=0.5)
    assert out["n_a"][0] == 0 and out["link_mask"][0] == 0
    assert out["r_contact"][0] == pytest.approx(-0.05, rel=1e-15)


def _pick(h, mesh, scene, links, model):
    """(env, frame link with a self-touched patch, link whose primitive touches
    it, object touching something)."""
    out = oracle.hand_forward(mesh, h, scene, links, model, rel32=False)
    O = scene.max_obj
    for e in range(scene.n_envs):
        c = out["contact_obj"][e]
        for k in range(mesh.n_patches):
            a, b = int(mesh.patch_offset[k]), int(mesh.patch_offset[k + 1])
            sel = c[a:b][c[a:b] >= O]
            if sel.size and (c >= 0).any() and ((c >= 0) & (c < O)).any():
                return e, int(h.patch_link[k]), int(sel[0]) - O, int(c[(c >= 0) & (c < O)][0])
    raise AssertionError("no env with self-contact and object contact")


@pytest.mark.parametrize("mode", [scenes.MODE_DECAY_ONLY, scenes.MODE_FULL])
def test_hand_pose_adjoint_vs_central_differences(oracle_lib, mode):
    h, mesh = art.hand()
    scene, links = art.grasp_scene(h, mesh, 24, seed=8)
    model = _model(mesh, mode)
    e, lf, lp, o = _pick(h, mesh, scene, links, model)
    sub, lk = scene.select([e]), links.select([e])
    w = np.random.default_rng(4).standard_normal((3, 1, mesh.n_nodes))
    g = oracle.hand_backward(mesh, h, sub, lk, model, w, rel32=False)
    checked = 0
    for target in (dict(link=lf), dict(link=lp), dict(obj=o)):
        fd, ok = oracle.hand_fd_gradients(mesh, h, sub, lk, model, w, env=0, **target)
        if "link" in target:
            G, T, R = g["grad_link_rot"][0, target["link"]], g["grad_link_trans"][0, target["link"]], lk.rot[0, target["link"]]
        else:
            G, T, R = g["grad_rot"][0, o], g["grad_trans"][0, o], sub.rot[0, o]
        tw = oracle.twist_from_grad_rot(G, R)
        for key, ad in (("trans", T), ("twist", tw)):
            okk = fd["ok_each"][key]
            scale = max(1.0, np.abs(ad).max())
            assert np.all(np.abs(fd[key][okk] - ad[okk]) <= 1e-6 * scale), (target, key, fd[key], ad)
            checked += int(okk.sum())
    assert checked >= 15
