"""The synthetic workloads have the properties their recipes state.

The benchmark hand (config 2) places each env's 1-3 objects by footprint so
that 5-30 % of the env's nodes are in contact; the generator holds no contact
arithmetic, so the band is checked here with the oracle's contact pass."""
import numpy as np

import scenes


def test_config2_contact_band(oracle_lib):
    mesh = scenes.hand_mesh(0)
    scene = scenes.hand_scene(mesh, 768, 1)
    _, _, na = oracle_lib.contact(mesh, scene)
    frac = na.sum(axis=1) / mesh.n_nodes
    inside = np.mean((frac >= 0.05) & (frac <= 0.30))
    print(f"active fraction: mean {frac.mean():.3f}, median {np.median(frac):.3f}, "
          f"p5 {np.percentile(frac, 5):.3f}, p95 {np.percentile(frac, 95):.3f}, in band {inside:.4f}")
    assert inside >= 0.95
    assert set(np.unique(scene.n_obj)) == {1, 2, 3}
    assert set(np.unique(scene.type[scene.n_obj[:, None] > np.arange(3)])) == {scenes.SPHERE, scenes.BOX,
                                                                                  scenes.CAPSULE}


def test_hand_envs_regenerate_alone():
    # env e draws from its own stream: a subset of envs regenerates identically
    mesh = scenes.hand_mesh(0)
    a = scenes.hand_scene(mesh, 40, 1)
    b = scenes.hand_scene(mesh, 12, 1)
    for f in ("n_obj", "type", "shape", "rot", "trans"):
        assert np.array_equal(getattr(a, f)[:12], getattr(b, f))


def test_rotations_are_proper():
    mesh = scenes.hand_mesh(0)
    sc = scenes.hand_scene(mesh, 64, 1)
    R = sc.rot.reshape(-1, 3, 3).astype(np.float64)
    live = (sc.n_obj[:, None] > np.arange(3)).ravel()
    R = R[live]
    assert np.allclose(R @ np.transpose(R, (0, 2, 1)), np.eye(3), atol=1e-6)
    assert np.allclose(np.linalg.det(R), 1.0, atol=1e-6)
