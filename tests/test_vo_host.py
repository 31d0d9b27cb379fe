"""Host logic of the sliding-window driver front end (paper_2208_04726_amd/
vo.py): pose composition checked against 4x4 homogeneous matrices, and the
trajectory assembly ("Keyframing", Sec. 3.3) on the pieces the driver oracle
keeps: every processed frame appears once, removed keyframes sit at their
stored relative pose from the keyframe before them, and frames still in the
window keep their window pose."""
import numpy as np

from oracle import vo_oracle as V
from paper_2208_04726_amd import synth
from paper_2208_04726_amd.vo import assemble_trajectory, compose


def _mat(p):
    x, y, z, w = p[3:] / np.linalg.norm(p[3:])
    R = np.array([[w * w + x * x - y * y - z * z, 2 * (x * y - w * z), 2 * (x * z + w * y)],
                  [2 * (x * y + w * z), w * w - x * x + y * y - z * z, 2 * (y * z - w * x)],
                  [2 * (x * z - w * y), 2 * (y * z + w * x), w * w - x * x - y * y + z * z]])
    M = np.eye(4)
    M[:3, :3], M[:3, 3] = R, p[:3]
    return M


def test_compose_is_the_matrix_product():
    rng = np.random.default_rng(3)
    for _ in range(20):
        a = np.concatenate([rng.normal(size=3), rng.normal(size=4)])
        b = np.concatenate([rng.normal(size=3), rng.normal(size=4)])
        a[3:] /= np.linalg.norm(a[3:])
        b[3:] /= np.linalg.norm(b[3:])
        np.testing.assert_allclose(_mat(compose(a, b)), _mat(a) @ _mat(b), atol=1e-12)


def test_trajectory_from_the_oracle_pieces():
    s = synth.make_stream(40, 8, seed=[9])
    o = V.StreamOracle(s, window=8, radius=3)
    for t in range(36):
        rec = o.step(t)
    removed = {f: (prev, rel) for f, prev, rel in o.removed}
    traj = assemble_trajectory(rec["kf"], rec["poses"], o.final, removed)
    assert sorted(traj) == list(range(36))
    assert len(removed) > 0 and len(o.final) > 0
    for f, (prev, rel) in removed.items():
        np.testing.assert_allclose(_mat(traj[f]), _mat(rel) @ _mat(traj[prev]), atol=1e-12)
    for f, p in zip(rec["kf"], rec["poses"]):
        np.testing.assert_array_equal(traj[f], p)
    for f, p in o.final.items():
        np.testing.assert_array_equal(traj[f], p)
