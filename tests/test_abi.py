"""The C-ABI library loads on the host and exports every function include/ld.h declares;
argument validation that happens before any HIP call works without a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ld.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ld_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_1807_02752_amd import ld
    if not os.path.exists(ld.LIB_PATH):
        pytest.fail("libld.so is not built: run __graft_entry__.build()")
    return ld.lib()


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert "ld_detect" in names and "ld_frame_create" in names and len(names) >= 12
    for n in names:
        assert hasattr(L, n), n
    from paper_1807_02752_amd import ld
    assert sorted(ld.EXPORTED) == names


def test_defaults_and_status_strings(L):
    from paper_1807_02752_amd import ld
    p = ld.params_default()
    assert (p.chi, p.tau_y_max, p.tau_x_max, p.tr_y, p.tr_x, p.varpi, p.edge_t, p.sigma_g) == \
        (25, 6, 5, 4.0, 16.0, 3.0, 100, 3.5)
    assert (p.eps_num, p.eps_den, p.nu, p.varsigma, p.n_hyp, p.max_rounds) == (99, 100, 1, 3, 64, 16)
    assert ld.ld_status_string(0) == "ok" and "invalid" in ld.ld_status_string(-1)


def test_invalid_arguments_rejected_before_any_device_call(L):
    from paper_1807_02752_amd import ld
    for args in [(4, 100, 1, 0, 32), (100, 4, 1, 0, 32), (5000, 100, 1, 0, 32), (100, 100, 0, 0, 32),
                 (100, 100, 1, 3, 32), (100, 100, 1, 0, 0), (100, 100, 1, 0, 2000)]:
        st, h = ld.ld_frame_create(*args)
        assert st == ld.LD_E_INVAL and not h.value
    bad = ld.params_default(n_hyp=65)
    assert ld.ld_frame_create(100, 100, 1, 0, 32, bad)[0] == ld.LD_E_INVAL
    bad = ld.params_default(tau_x_max=6)
    assert ld.ld_frame_create(100, 100, 1, 0, 32, bad)[0] == ld.LD_E_INVAL
    assert L.ld_frame_create(100, 100, 1, 0, 32, None, None) == ld.LD_E_INVAL
    assert ld.ld_vdisp(None, None, 0, None, None, None, None, None) == ld.LD_E_INVAL
    assert ld.ld_detect(None, None, 0, None, 0, None, None, None, None, None) == ld.LD_E_INVAL
    assert ld.ld_sync(None) == ld.LD_E_INVAL
    assert ld.ld_bilateral(None, None, 0, None, 0, 5, 300.0, 0.3, 0, None) == ld.LD_E_INVAL
    assert ld.ld_stereo(None, None, 0, None, 0, 3, 1, 3, None, 0, None, None, None) == ld.LD_E_INVAL
    assert ld.ld_frame_destroy(None) == ld.LD_OK


def test_product_path_never_touches_the_oracle():
    pkg = os.path.join(ROOT, "paper_1807_02752_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, fn
                assert "ldref" not in txt, fn


def test_server_config_validation_without_device(L):
    from paper_1807_02752_amd import ld
    for bad in [dict(classes=[]), dict(classes=[(4, 96, 0, 48, 4)]), dict(classes=[(320, 96, 7, 48, 4)]),
                dict(classes=[(320, 96, 0, 48, 0)]), dict(classes=[(320, 96, 0, 48, 4)], inflight=0),
                dict(classes=[(320, 96, 0, 48, 4)], max_queue=0)]:
        classes = bad.pop("classes")
        cfg = ld.server_config(classes, **bad)
        st, h = ld.ld_server_create(cfg)
        assert st == ld.LD_E_INVAL and not h.value
    assert ld.ld_server_destroy(None) == ld.LD_OK
    assert ld.ld_server_submit(None, 0, 0, None, 0, None, 0)[0] == ld.LD_E_INVAL


def test_noalloc_argument_checks_without_device(L):
    """ld_detect_noalloc validates sizes and rejects a scratch need beyond its fixed array
    before any HIP call (the pointers below are never dereferenced)."""
    from paper_1807_02752_amd import ld
    fake = C.c_void_p(1 << 20)
    args = lambda w, h, b, fmt, dm: (w, h, b, fmt, dm, None, fake, w, fake, w * 4, None, None, fake, None, None)
    assert ld.ld_detect_noalloc(*args(4, 375, 1, ld.LD_DISP_F32, 128)) == ld.LD_E_INVAL
    assert ld.ld_detect_noalloc(*args(1242, 375, 0, ld.LD_DISP_F32, 128)) == ld.LD_E_INVAL
    assert ld.ld_detect_noalloc(*args(1242, 375, 1, 5, 128)) == ld.LD_E_INVAL
    assert ld.ld_detect_noalloc(*args(1242, 375, 11, ld.LD_DISP_F32, 128)) == ld.LD_E_NOMEM
    assert ld.ld_detect_noalloc(*args(1920, 1080, 3, ld.LD_DISP_F32, 255)) == ld.LD_E_NOMEM
    no_lanes = list(args(1242, 375, 1, ld.LD_DISP_F32, 128))
    no_lanes[12] = None
    assert ld.ld_detect_noalloc(*no_lanes) == ld.LD_E_INVAL
