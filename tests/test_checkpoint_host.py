"""Host-side parts of the stage checkpoints and of the launch-fault hook:
stage discovery in a checkpoint directory, refusal of another build's
files, and arming the hook by call and by environment (no GPU involved)."""
import os
import subprocess
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
import paper_1307_7852_amd as K  # noqa: E402
from paper_1307_7852_amd import checkpoint as C  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _touch(d, name):
    np.save(os.path.join(d, name), np.zeros(3, dtype=np.uint32))


def test_stage_discovery(tmp_path):
    d = str(tmp_path)
    assert C.checkpoint_stages(d) == {"divisions": [], "perms": [], "merged": False, "rounds": 0}
    for f in ["perm_0.npy", "leaf_off_0.npy", "ids_0.npy", "dist_0.npy", "perm_1.npy", "leaf_off_1.npy",
              "perm_2.npy", "ids_3.npy", "merged_ids.npy", "round_1_ids.npy", "round_1_dist.npy",
              "round_3_ids.npy", "round_3_dist.npy"]:
        _touch(d, f)
    open(os.path.join(d, "merged_dist.npy.part"), "wb").close()   # an unfinished write is no stage
    s = C.checkpoint_stages(d)
    # division 0 complete; division 1 partitioned; perm_2 lacks its offsets and
    # ids_3 its distances; rounds count up to the first gap
    assert s == {"divisions": [0], "perms": [1], "merged": False, "rounds": 1}
    _touch(d, "merged_dist.npy")
    assert C.checkpoint_stages(d)["merged"]


def test_refuses_other_build(tmp_path):
    d = str(tmp_path / "ck")
    X = torch.from_numpy(np.arange(64 * 8, dtype=np.float32).reshape(64, 8))
    p = K.Params(n=64, d=8, k=4, T=2, leaf_max=16, rounds=1, seed=5)
    # the directory records these parameters and the data's digest, then the host tensor is refused
    with pytest.raises(ValueError, match="device tensor"):
        C.build_resumable(X, p, d)
    assert os.path.exists(os.path.join(d, "meta.json"))
    with pytest.raises(ValueError, match="another build"):
        C.build_resumable(X, K.Params(n=64, d=8, k=4, T=3, leaf_max=16, rounds=1, seed=5), d)
    X2 = X.clone()
    X2[5, 3] += 1.0
    with pytest.raises(ValueError, match="another build"):
        C.build_resumable(X2, p, d)
    with pytest.raises(ValueError, match="device tensor"):
        C.build_resumable(X, p, d)
    with pytest.raises(ValueError, match="shape"):
        C.build_resumable(X[:, :4].contiguous(), p, d)
    with pytest.raises(ValueError, match="effective-rate"):
        C.build_resumable(X, K.Params(n=64, d=8, k=4, T=2, leaf_max=16, rate_permille=50), d)


def test_fault_hook_arm_disarm():
    assert K.inject_fault(1) == 0
    assert K.inject_fault(1) == 1
    assert K.inject_fault(0) == 1
    assert K.inject_fault(0) == 0
    with pytest.raises(K.KnngError, match="KNNG_EINVAL"):
        K.inject_fault(2)
    assert K.inject_fault(0) == 0


@pytest.mark.parametrize("value,armed", [("launch", 1), ("", 0), ("other", 0)])
def test_fault_hook_from_environment(value, armed):
    env = dict(os.environ)
    env["KNNG_FAULT"] = value
    out = subprocess.run([sys.executable, "-c", "import paper_1307_7852_amd as K; print(K.inject_fault(0))"],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == str(armed)
