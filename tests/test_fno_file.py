"""FNO weight files: host-side validation (CPU) and the save/load round trip (GPU).

The CPU tests write a file in the documented layout of include/parareal.h
(96-byte header, FNV-1a 64 checksum over the first 80 header bytes and the
weights, then the FP32 weights) and check that pr_fno_check_file accepts it
and rejects every corruption with PR_EMODEL.
"""
import struct

import numpy as np
import pytest

from paper_2404_02521_amd import _lib as L
from paper_2404_02521_amd import fno as F

ARCH = (64, 32, 12, 4, 7, 64, 128)


def fnv1a(data: bytes, h: int = 1469598103934665603) -> int:
    for b in data:
        h ^= b
        h = (h * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return h


def make_file(path, weights, base=L.PR_FNO_BASE_IDENTITY, prec=L.PR_FNO_FP32, scale=0.015625,
              thash=0x1234, version=1, arch=ARCH, count=None, magic=b"PRFNOW01", fix_sum=True,
              trailing=b""):
    w = np.ascontiguousarray(weights, dtype="<f4").tobytes()
    count = len(weights) if count is None else count
    head = magic + struct.pack("<II", version, 96) + struct.pack("<7i", *arch)
    head += struct.pack("<iii", base, prec, 0) + struct.pack("<d", scale)
    head += struct.pack("<QQ", count, thash)
    assert len(head) == 80
    s = fnv1a(w, fnv1a(head)) if fix_sum else 0
    path.write_bytes(head + struct.pack("<QQ", s, 0) + w + trailing)


@pytest.fixture(scope="module")
def weights():
    n = F.param_count()
    return np.random.default_rng(5).standard_normal(n).astype(np.float32) * 0.05


def status_of(path):
    try:
        F.check_file(str(path))
        return L.PR_OK
    except L.PararealError as e:
        return e.status


def test_valid_file_accepted(tmp_path, weights):
    p = tmp_path / "w.prfno"
    make_file(p, weights)
    info = F.check_file(str(p))
    assert info == dict(version=1, base=L.PR_FNO_BASE_IDENTITY, precision=L.PR_FNO_FP32,
                        out_scale=0.015625, param_count=len(weights), train_hash=0x1234)


def test_corrupted_files_rejected(tmp_path, weights):
    cases = {
        "flipped weight byte": None,
        "truncated": None,
        "wrong magic": dict(magic=b"PRFNOX01"),
        "wrong version": dict(version=2),
        "other width": dict(arch=(64, 64, 12, 4, 7, 64, 128)),
        "wrong count": dict(count=len(weights) - 1),
        "bad checksum": dict(fix_sum=False),
        "bad base": dict(base=9),
        "bad precision": dict(prec=3),
        "bad scale": dict(scale=-1.0),
        "trailing bytes": dict(trailing=b"\0"),
    }
    for name, kw in cases.items():
        p = tmp_path / (name.replace(" ", "_") + ".prfno")
        make_file(p, weights, **(kw or {}))
        if name == "flipped weight byte":
            b = bytearray(p.read_bytes())
            b[96 + 1000] ^= 0x40
            p.write_bytes(bytes(b))
        if name == "truncated":
            p.write_bytes(p.read_bytes()[:-4])
        assert status_of(p) == L.PR_EMODEL, name
    w = weights.copy()
    w[7] = np.nan
    p = tmp_path / "nan.prfno"
    make_file(p, w)   # checksum consistent, but a weight is not finite
    assert status_of(p) == L.PR_EMODEL
    assert status_of(tmp_path / "missing.prfno") == L.PR_EMODEL
    (tmp_path / "empty.prfno").write_bytes(b"")
    assert status_of(tmp_path / "empty.prfno") == L.PR_EMODEL


@pytest.mark.gpu
def test_save_load_round_trip(tmp_path):
    import torch
    from helpers import say
    from paper_2404_02521_amd.train import init_params
    from synthetic import fno_batch
    say("fno save/load round trip")
    a = F.Fno(max_batch=4, out_scale=0.5)
    a.set_params(init_params(3))
    p = tmp_path / "a.prfno"
    a.save(str(p), train_hash=77)
    info = F.check_file(str(p))
    assert info["train_hash"] == 77 and info["out_scale"] == 0.5
    b = F.Fno(max_batch=4, out_scale=0.5)
    b.set_params(init_params(4))
    before = b.params().clone()
    assert b.load(str(p))["train_hash"] == 77
    assert torch.equal(a.params(), b.params())
    w, meta = fno_batch(11, 4)
    w = torch.from_numpy(w).cuda()
    meta = torch.from_numpy(meta).cuda()
    assert torch.equal(a.forward(w, meta), b.forward(w, meta))
    # a handle of another configuration refuses the file and keeps its weights
    c = F.Fno(max_batch=4, out_scale=0.25)
    c.set_params(before)
    with pytest.raises(L.PararealError) as e:
        c.load(str(p))
    assert e.value.status == L.PR_EMODEL
    assert torch.equal(c.params(), before)
    # a corrupted file leaves the handle unchanged
    raw = bytearray(p.read_bytes())
    raw[200] ^= 1
    p.write_bytes(bytes(raw))
    with pytest.raises(L.PararealError) as e:
        b.load(str(p))
    assert e.value.status == L.PR_EMODEL
    assert torch.equal(b.params(), a.params())
    for h in (a, b, c):
        h.close()
