"""Host-side logic of the learned initialiser's training data: the batched
draw of rigid offsets."""
import numpy as np

from paper_1611_07289_amd import synth


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
