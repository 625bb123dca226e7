"""Checkpoint round trip on the host (no GPU needed): the active set with
both Adam moments and rate factors, named pose tensors and anchors' host
blocks come back bit for bit, with their keyframes, locations and step."""
import numpy as np
import torch

from paper_2506_05558_amd import checkpoint, gsmi
from paper_2506_05558_amd.scalable import ActiveSet, Anchor


def _gauss(rng, n, d):
    f = lambda *s: torch.tensor(rng.standard_normal(s).astype(np.float32))
    return gsmi.Gaussians(f(3, n), f(3, n), f(4, n), f(n), f((d + 1) ** 2, 3, n))


def test_round_trip(tmp_path):
    rng = np.random.default_rng(0)
    n, d = 1001, 3
    act = ActiveSet(_gauss(rng, n, d), _gauss(rng, n, d), _gauss(rng, n, d),
                    torch.tensor(rng.random(n).astype(np.float32)), [3, 4, 7])
    act.g.means[0, 5] = float("nan")  # values are copied, not interpreted
    poses = {"x6": torch.tensor(rng.standard_normal((8, 9)).astype(np.float32)),
             "x6_m": torch.zeros((8, 9)), "d_pose": torch.tensor(rng.standard_normal((8, 12)))}
    anchors = [Anchor(np.array([1.0, 2.0, 3.5]), 77, 0, [0, 1], torch.tensor(rng.integers(0, 255, 4096, np.uint8)),
                      None),
               Anchor(np.array([-1.0, 0.25, 9.0]), 12, 3, [5], torch.tensor(rng.integers(0, 255, 300, np.uint8)),
                      None)]
    path = str(tmp_path / "ckpt.safetensors")
    checkpoint.save(path, act, poses, anchors, step=42, extra={"note": "round trip"})
    out = checkpoint.load(path, device="cpu")
    assert out["step"] == 42 and out["extra"] == {"note": "round trip"}
    b = out["active"]
    for x, y in zip(act.tensors(), b.tensors()):
        assert x.dtype == y.dtype and x.shape == y.shape
        assert np.array_equal(x.numpy().view(np.uint32), y.numpy().view(np.uint32))
    assert b.keyframes == [3, 4, 7] and b.g.sh_degree == 3
    for k, v in poses.items():
        assert torch.equal(v, out["poses"][k]) and v.dtype == out["poses"][k].dtype
    assert len(out["anchors"]) == 2
    for a, c in zip(anchors, out["anchors"]):
        assert torch.equal(a.host, c.host) and a.n == c.n and a.sh_degree == c.sh_degree
        assert a.keyframes == c.keyframes and np.array_equal(a.location, c.location)


def test_rejects_foreign_file(tmp_path):
    from safetensors.torch import save_file
    path = str(tmp_path / "other.safetensors")
    save_file({"x": torch.zeros(3)}, path, metadata={"gsmi": '{"format": "something-else"}'})
    try:
        checkpoint.load(path, device="cpu")
    except ValueError as e:
        assert "not a" in str(e)
    else:
        raise AssertionError("a foreign file was accepted")
