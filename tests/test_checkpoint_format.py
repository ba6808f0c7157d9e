"""The network checkpoint file (ld_cnn_save / ld_cnn_load): its layout, read back by the Python
reader, and the checks ld_cnn_load makes before any device call (no GPU needed)."""
import json
import os

import numpy as np
import pytest


@pytest.fixture(scope="module")
def ld():
    from paper_1807_02752_amd import ld as m
    if not os.path.exists(m.LIB_PATH):
        pytest.fail("libld.so is not built: run __graft_entry__.build()")
    m.lib()
    return m


def _write(path, header, arrays, extra=b""):
    with open(path, "wb") as fp:
        fp.write((json.dumps(header) + "\n").encode())
        for a in arrays:
            fp.write(np.asarray(a, "<f4").tobytes())
        fp.write(extra)


def _header(ld, **kw):
    h = {"format": "ld_cnn_checkpoint", "version": 1, "params": ld.LD_CNN_PARAMS, "step": 7, "dtype": "float32",
         "arrays": ["master", "adam_m", "adam_v"],
         "config": {"n_bands": 1, "theta": 0.5, "delta_x": 112, "dilate": -1, "min_votes": 8, "max_batch": 32,
                    "max_width": 1920, "seed_ransac": 0}}
    h.update(kw)
    return h


def test_reader_round_trip(ld, tmp_path):
    rng = np.random.default_rng(0)
    arrays = [rng.standard_normal(ld.LD_CNN_PARAMS).astype(np.float32) for _ in range(3)]
    p = str(tmp_path / "a.ckpt")
    _write(p, _header(ld), arrays)
    header, got = ld.read_checkpoint(p)
    assert header["step"] == 7
    for name, a in zip(ld.CKPT_FIELDS, arrays):
        assert np.array_equal(got[name], a)
    assert os.path.getsize(p) == len(json.dumps(_header(ld))) + 1 + 3 * 4 * ld.LD_CNN_PARAMS


@pytest.mark.parametrize("case", ["missing", "truncated", "trailing", "version", "params", "format", "step"])
def test_load_rejects_bad_files_before_the_device(ld, tmp_path, case):
    p = str(tmp_path / "b.ckpt")
    arrays = [np.zeros(ld.LD_CNN_PARAMS, np.float32)] * 3
    if case == "missing":
        p = str(tmp_path / "none.ckpt")
    elif case == "truncated":
        _write(p, _header(ld), arrays[:2])
    elif case == "trailing":
        _write(p, _header(ld), arrays, extra=b"\0")
    elif case == "version":
        _write(p, _header(ld, version=2), arrays)
    elif case == "params":
        _write(p, _header(ld, params=ld.LD_CNN_PARAMS + 1), arrays)
    elif case == "format":
        _write(p, _header(ld, format="other"), arrays)
    elif case == "step":
        _write(p, _header(ld, step=-1), arrays)
    st, h = ld.ld_cnn_load(p)
    assert st == ld.LD_E_INVAL and not h.value
    assert ld.ld_cnn_save(None, p) == ld.LD_E_INVAL
