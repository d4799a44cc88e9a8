"""Pins of the dense verification reference (oracle/verify.py)."""
import numpy as np

from oracle import Params
from oracle.frames import prepare_frame
from oracle.verify import verify_direction, verify_pairs
from synth import make_chunk


def test_frame_against_itself():
    """A frame verified against an identical copy at the same pose: every pixel with
    a valid normal and finite intensity associates with itself at zero error."""
    pr = make_chunk(num_frames=3, noise=False, outlier_rate=0.0)
    prm = Params()
    f = prepare_frame(pr.depth[1], pr.intensity[1], pr.intrinsics, prm)
    e, n, _ = verify_direction(f, f, pr.intensity[1], pr.intensity[1], pr.gt_poses[1], pr.gt_poses[1], pr.intrinsics,
                            prm, 0.1)
    assert n == int(f.normal_ok.sum()) and n > 0
    assert e < 1e-9   # the relative pose of a pose with itself is the identity up to rounding


def test_ground_truth_valid_and_misaligned_invalid():
    pr = make_chunk(num_frames=5, noise=False, outlier_rate=0.0)
    prm = Params()
    pairs = [(0, 1), (1, 2), (0, 3), (2, 4)]
    st, ok, _ = verify_pairs(pr.depth, pr.intensity, pr.intrinsics, pairs, pr.gt_poses, prm)
    assert ok.all()
    # at ground truth only the nearest-pixel lookup at 80x60 leaves an error (about a centimetre)
    assert (st[:, 0] / st[:, 1]).max() < 0.02 and (st[:, 2] / st[:, 3]).max() < 0.02
    bad = pr.gt_poses.copy()
    bad[3, :3, 3] += np.array([0.2, 0.0, 0.0])   # frame 3 moved by 20 cm
    st2, ok2, _ = verify_pairs(pr.depth, pr.intensity, pr.intrinsics, pairs, bad, prm)
    assert ok2[[0, 1, 3]].all() and not ok2[2]
    assert st2[2, 0] / st2[2, 1] > 0.075


def test_photoconsistency_term():
    """Intensities of frame j farther than tau_c from all of frame i's reject every
    association of the pair; an unbounded tau_c keeps at least as many."""
    pr = make_chunk(num_frames=2, noise=False, outlier_rate=0.0)
    prm = Params()
    inten = pr.intensity.copy()
    st0, _, _ = verify_pairs(pr.depth, inten, pr.intrinsics, [(0, 1)], pr.gt_poses, prm)
    inten[1] = 2.0   # farther than tau_c from every intensity of frame 0 (all in [0, 1])
    st1, ok1, _ = verify_pairs(pr.depth, inten, pr.intrinsics, [(0, 1)], pr.gt_poses, prm)
    assert st1[0, 1] == 0 and st1[0, 3] == 0 and not ok1[0]
    inten[1] = pr.intensity[1] + 0.0
    st2, _, _ = verify_pairs(pr.depth, inten, pr.intrinsics, [(0, 1)], pr.gt_poses, prm, tau_c=10.0)
    assert st2[0, 1] >= st0[0, 1] and st2[0, 3] >= st0[0, 3]
