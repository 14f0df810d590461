"""Host-side logic of the learned initialiser: the target maps between motion
offsets and network targets."""
import types

import numpy as np

from paper_1611_07289_amd import learned, pvr, synth


def _fake_plan():
    c = np.array([10.0, 20.0, 30.0])
    stacks = [synth.make_stack(c, *fr, 32, 32, 8, (1, 1), 4.0, (1.0, 1.0, 4.0))
              for fr in synth.orthogonal_frames([30.0])]
    P = synth.square_patches(stacks, 16, 8)
    S = [types.SimpleNamespace(pix2world=np.asarray(st.pix2world, float).reshape(-1)[:12])
         for st in stacks]
    tab = np.ascontiguousarray(np.asarray(P.table(), dtype=np.int32))
    Q = (pvr.Patch * P.M).from_buffer_copy(tab.tobytes())
    return types.SimpleNamespace(_s=S, _p=Q, M=P.M), stacks, P


def test_target_maps_are_inverse_pairs_in_the_stack_frame():
    plan, stacks, P = _fake_plan()
    A, Ai = learned.target_maps(plan)
    eye = np.eye(6, dtype=np.float32)
    assert np.allclose(A @ Ai, eye, atol=1e-5)
    rho = 0.5 * np.hypot(15.0, 15.0)
    for i in range(plan.M):
        st = stacks[P.stack[i]]
        L = np.asarray(st.pix2world, float).reshape(3, 4)[:, :3]
        n = L[:, 2] / np.linalg.norm(L[:, 2])
        # a translation along the slice normal is the third translation target
        off = np.r_[0, 0, 0, n]
        assert np.allclose(A[i] @ off, [0, 0, 0, 0, 0, 1], atol=1e-6)
        # a small rotation about the normal is an in-plane rotation, scaled by rho
        off = np.r_[1e-3 * n, 0, 0, 0]
        assert np.allclose(A[i] @ off, [0, 0, 1e-3 * rho, 0, 0, 0], atol=1e-6)


def test_batched_motion_draws_follow_the_motion_distribution():
    """The vectorised draw has the distribution of the per-patch one: angle
    U[0, max] about a uniform axis (recovered from the Euler angles), shift
    uniform in the ball."""
    from scipy.spatial.transform import Rotation
    th = synth.random_motion_batch(20000, 10.0, 5.0, 3)
    R = Rotation.from_euler("xyz", th[:, :3]).as_matrix()  # R = Rz Ry Rx
    ang = np.degrees(np.arccos(np.clip((np.trace(R, axis1=1, axis2=2) - 1) / 2, -1, 1)))
    assert ang.max() <= 10.0 + 1e-9 and abs(ang.mean() - 5.0) < 0.1
    r = np.linalg.norm(th[:, 3:], axis=1)
    assert r.max() <= 5.0 + 1e-12
    # uniform in the ball: P(r <= 5 s) = s^3
    assert abs(np.mean(r <= 2.5) - 0.125) < 0.01
    ref = synth.random_motion(2000, 10.0, 5.0, 4)
    Rr = Rotation.from_euler("xyz", ref[:, :3]).as_matrix()
    ang_r = np.degrees(np.arccos(np.clip((np.trace(Rr, axis1=1, axis2=2) - 1) / 2, -1, 1)))
    assert abs(ang_r.mean() - ang.mean()) < 0.3
