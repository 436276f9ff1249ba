"""Host-side checks of the C ABI: the library loads, exports every declared
function, and rejects bad arguments before touching the GPU."""
import ctypes
import re

import pytest

from paper_1902_09733_amd import _abi


@pytest.fixture(scope="module")
def lib():
    return _abi.lib()


def test_exports_every_declared_function(lib):
    names = _abi.header_functions()
    assert {"bp_cost_volume", "bp_run", "bp_upsample", "bp_backward"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings(lib):
    for code in (0, -1, -2, -3, -4):
        assert lib.bp_status_string(code)
    assert lib.bp_status_string(0) == b"ok"


def _prob(w=16, h=8, L=8, cost=1):
    p = (_abi.BpProblem * 1)()
    p[0].width, p[0].height, p[0].num_labels = w, h, L
    p[0].cost = cost
    return p


def _params(**kw):
    d = dict(levels=1, iters_per_level=4, lambda_=10.0, tau=2.0, msg_dtype=0, temperature=0.5,
             checkpoint_every=0, variant=0, pm_from=-1)
    d.update(kw)
    return _abi.BpParams(**d)


def test_workspace_size_grows_and_rejects(lib):
    p = _params()
    a = lib.bp_workspace_size(_prob(16, 8, 8), 1, ctypes.byref(p))
    b = lib.bp_workspace_size(_prob(32, 8, 8), 1, ctypes.byref(p))
    assert 0 < a < b and a % 256 == 0
    assert lib.bp_workspace_size(_prob(16, 8, 1), 1, ctypes.byref(p)) == 0      # L < 2
    assert lib.bp_workspace_size(_prob(16, 8, 257), 1, ctypes.byref(p)) == 0    # L > 256
    assert lib.bp_workspace_size(_prob(0, 8, 8), 1, ctypes.byref(p)) == 0
    bad = _params(tau=0.0)
    assert lib.bp_workspace_size(_prob(), 1, ctypes.byref(bad)) == 0
    p2 = _params(levels=3, msg_dtype=1)
    assert lib.bp_workspace_size(_prob(16, 8, 8), 1, ctypes.byref(p2)) > 0


def _pair(**kw):
    d = dict(left=256, right=512, channels=3, downsample=4, row_stride_bytes=16 * 4 * 3, data_trunc=20.0,
             rgb_mode=0)
    d.update(kw)
    return _abi.BpPair(**d)


def test_pair_source_validation(lib):
    """A problem without a cost volume needs a valid pair; the workspace then
    also holds the packed downsampled pair (2 x W x H words)."""
    p = _params()
    with_cost = lib.bp_workspace_size(_prob(16, 8, 8), 1, ctypes.byref(p))
    pr = _pair()
    q = _prob(16, 8, 8, cost=0)
    q[0].pair = ctypes.pointer(pr)
    with_pair = lib.bp_workspace_size(q, 1, ctypes.byref(p))
    assert with_pair >= with_cost + 2 * 16 * 8 * 4
    assert lib.bp_workspace_size(_prob(16, 8, 8, cost=0), 1, ctypes.byref(p)) == 0        # neither
    for bad in (dict(left=0), dict(right=0), dict(channels=2), dict(downsample=0),
                dict(row_stride_bytes=16 * 4 * 3 - 1), dict(data_trunc=-1.0), dict(data_trunc=float("nan")),
                dict(rgb_mode=2)):
        pb = _pair(**bad)
        qb = _prob(16, 8, 8, cost=0)
        qb[0].pair = ctypes.pointer(pb)
        assert lib.bp_workspace_size(qb, 1, ctypes.byref(p)) == 0, bad
        st = lib.bp_run(qb, 1, ctypes.byref(p), ctypes.c_void_p(256), 1 << 20, None, 0, None)
        assert st == _abi.BP_ERR_INVALID_ARGUMENT, bad


@pytest.mark.parametrize("kw,expect", [
    (dict(lambda_=-1.0), _abi.BP_ERR_INVALID_ARGUMENT),
    (dict(tau=0.0), _abi.BP_ERR_INVALID_ARGUMENT),
    (dict(levels=0), _abi.BP_ERR_INVALID_ARGUMENT),
    (dict(iters_per_level=-1), _abi.BP_ERR_INVALID_ARGUMENT),
    (dict(msg_dtype=7), _abi.BP_ERR_INVALID_ARGUMENT),
    (dict(pm_from=5), _abi.BP_ERR_INVALID_ARGUMENT),
    (dict(pm_from=-2), _abi.BP_ERR_INVALID_ARGUMENT),
])
def test_run_rejects_bad_params(lib, kw, expect):
    p = _params(**kw)
    st = lib.bp_run(_prob(), 1, ctypes.byref(p), ctypes.c_void_p(256), 1 << 20, None, 0, None)
    assert st == expect


def test_run_rejects_bad_problems(lib):
    p = _params()
    ws = ctypes.c_void_p(256)
    assert lib.bp_run(_prob(cost=0), 1, ctypes.byref(p), ws, 1 << 20, None, 0, None) == _abi.BP_ERR_INVALID_ARGUMENT
    assert lib.bp_run(_prob(L=1), 1, ctypes.byref(p), ws, 1 << 20, None, 0, None) == _abi.BP_ERR_UNSUPPORTED
    assert lib.bp_run(_prob(L=300), 1, ctypes.byref(p), ws, 1 << 20, None, 0, None) == _abi.BP_ERR_UNSUPPORTED
    assert lib.bp_run(_prob(), 1, ctypes.byref(p), ctypes.c_void_p(100), 1 << 20, None, 0, None) == \
        _abi.BP_ERR_INVALID_ARGUMENT   # misaligned workspace
    assert lib.bp_run(_prob(), 1, ctypes.byref(p), ws, 16, None, 0, None) == _abi.BP_ERR_WORKSPACE_TOO_SMALL
    assert lib.bp_run(_prob(), 0, ctypes.byref(p), ws, 1 << 20, None, 0, None) == _abi.BP_ERR_INVALID_ARGUMENT
    soft = _prob()
    soft[0].soft_disparity = 256
    p0 = _params(temperature=0.0)
    assert lib.bp_run(soft, 1, ctypes.byref(p0), ws, 1 << 20, None, 0, None) == _abi.BP_ERR_INVALID_ARGUMENT


def test_cost_volume_rejects(lib):
    v = ctypes.c_void_p(256)
    f = lib.bp_cost_volume
    assert f(None, v, 8, 8, 1, 8, 1, 4, 20.0, 0, v, None) == _abi.BP_ERR_INVALID_ARGUMENT
    assert f(v, v, 8, 8, 2, 16, 1, 4, 20.0, 0, v, None) == _abi.BP_ERR_INVALID_ARGUMENT   # channels
    assert f(v, v, 8, 8, 1, 4, 1, 4, 20.0, 0, v, None) == _abi.BP_ERR_INVALID_ARGUMENT    # stride
    assert f(v, v, 10, 8, 1, 10, 4, 4, 20.0, 0, v, None) == _abi.BP_ERR_INVALID_ARGUMENT  # s must divide
    assert f(v, v, 8, 8, 1, 8, 1, 0, 20.0, 0, v, None) == _abi.BP_ERR_INVALID_ARGUMENT    # labels
    assert f(v, v, 8, 8, 1, 8, 1, 4, -1.0, 0, v, None) == _abi.BP_ERR_INVALID_ARGUMENT    # trunc
    assert f(v, v, 8, 8, 1, 8, 1, 4, 20.0, 2, v, None) == _abi.BP_ERR_INVALID_ARGUMENT    # rgb mode


def test_upsample_rejects(lib):
    v = ctypes.c_void_p(256)
    f = lib.bp_upsample
    assert f(v, 4, 4, v, 16, 12, 3, 48, 8.0, 12.0, -1, v, None) == _abi.BP_ERR_INVALID_ARGUMENT  # scales differ
    assert f(v, 4, 4, v, 16, 16, 3, 48, 0.0, 12.0, -1, v, None) == _abi.BP_ERR_INVALID_ARGUMENT  # sigma_s
    assert f(v, 4, 4, v, 16, 16, 3, 48, 8.0, 12.0, 9, v, None) == _abi.BP_ERR_UNSUPPORTED
    assert f(v, 4, 4, v, 16, 16, 3, 47, 8.0, 12.0, -1, v, None) == _abi.BP_ERR_INVALID_ARGUMENT  # stride
    big = 1 << 20
    assert f(v, big // 4, 4, v, big, 16, 1, big, 8.0, 12.0, -1, v, None) == _abi.BP_ERR_UNSUPPORTED  # width


def test_variant_counts(lib):
    assert lib.bp_variant_count(1) == 0
    for L in (2, 16, 32, 48, 64, 96, 128, 256):
        assert lib.bp_variant_count(L) >= 1


def test_tune_table_loading(lib, tmp_path):
    t = tmp_path / "t.txt"
    t.write_text("# comment\n676 380 64 0 5 0 1 900.0\nnot a line\n")
    assert lib.bp_load_tune_table(str(t).encode()) == 0
    assert lib.bp_load_tune_table(str(tmp_path / "missing.txt").encode()) == _abi.BP_ERR_INVALID_ARGUMENT
    assert lib.bp_load_tune_table(None) == 0


def test_upsample_points_validation(lib):
    """bp_upsample_points rejects a missing or degenerate camera before any launch."""
    cam_ok = dict(baseline=0.5, focal=3e-3, du=1.5e-6, dv=1.5e-6, u0=10.0, v0=8.0)
    args = lambda cam, pts: (ctypes.c_void_p(256), 4, 4, ctypes.c_void_p(512), 16, 16, 1, 16, 8.0, 12.0, -1,
                             cam, None, pts, None)
    assert lib.bp_upsample_points(*args(None, ctypes.c_void_p(1024))) == _abi.BP_ERR_INVALID_ARGUMENT
    c = _abi.BpCamera(**cam_ok)
    assert lib.bp_upsample_points(*args(ctypes.byref(c), None)) == _abi.BP_ERR_INVALID_ARGUMENT
    for bad in (dict(focal=0.0), dict(du=-1.0), dict(dv=0.0), dict(u0=float("inf")), dict(baseline=float("nan"))):
        cb = _abi.BpCamera(**dict(cam_ok, **bad))
        assert lib.bp_upsample_points(*args(ctypes.byref(cb), ctypes.c_void_p(1024))) == \
            _abi.BP_ERR_INVALID_ARGUMENT, bad


def test_icp_validation(lib):
    """bp_icp rejects bad sizes, pointers, dmax and workspace before any launch."""
    assert lib.bp_icp_workspace_size(-1, 10) == 0 and lib.bp_icp_workspace_size(10, -1) == 0
    n, m = 1000, 2000
    nb = lib.bp_icp_workspace_size(n, m)
    assert nb > 0 and lib.bp_icp_workspace_size(n, 4 * m) > nb
    P = ctypes.c_void_p
    good = dict(src=P(256), n=n, dst=P(512), m=m, pose_in=P(768), iters=5, dmax=1.0, pose_out=P(1024),
                rms=None, pairs=None, corr=None, ws=P(4096), nb=nb, stream=None)
    call = lambda **kw: lib.bp_icp(*dict(good, **kw).values())
    for bad in (dict(n=-1), dict(m=-1), dict(iters=-1), dict(src=None), dict(dst=None), dict(pose_in=None),
                dict(pose_out=None), dict(dmax=0.0), dict(dmax=-1.0), dict(dmax=float("nan")),
                dict(dmax=float("inf")), dict(ws=None), dict(ws=P(4096 + 8))):
        assert call(**bad) == _abi.BP_ERR_INVALID_ARGUMENT, bad
    assert call(nb=nb - 1) == _abi.BP_ERR_WORKSPACE_TOO_SMALL


def test_noalloc_size_and_checks_before_any_device_call(lib):
    """bp_run_noalloc rejects bad arguments and problems larger than its fixed
    array on the host, before it touches a device (so these run without one)."""
    src = open(_abi.HEADER).read()
    m = re.search(r"#define BP_NOALLOC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", src)
    assert m and int(m.group(1)) << int(m.group(2)) == _abi.BP_NOALLOC_SCRATCH_BYTES
    p = _params()
    assert lib.bp_run_noalloc(_prob(), 0, ctypes.byref(p), None, 0, None) == _abi.BP_ERR_INVALID_ARGUMENT
    assert lib.bp_run_noalloc(_prob(L=300), 1, ctypes.byref(p), None, 0, None) == _abi.BP_ERR_UNSUPPORTED
    bad = _params(tau=0.0)
    assert lib.bp_run_noalloc(_prob(), 1, ctypes.byref(bad), None, 0, None) == _abi.BP_ERR_INVALID_ARGUMENT
    # 1352 x 760 x 128 labels, six levels: about 3.3 GB of workspace.
    big = _prob(1352, 760, 128)
    p6 = _params(levels=6)
    assert lib.bp_workspace_size(big, 1, ctypes.byref(p6)) > _abi.BP_NOALLOC_SCRATCH_BYTES
    assert lib.bp_run_noalloc(big, 1, ctypes.byref(p6), None, 0, None) == _abi.BP_ERR_WORKSPACE_TOO_SMALL
    # The benchmarked 676 x 380 x 64 five-level problem from a pair fits.
    pr = _pair(row_stride_bytes=2704 * 3)
    q = _prob(676, 380, 64, cost=0)
    q[0].pair = ctypes.pointer(pr)
    assert 0 < lib.bp_workspace_size(q, 1, ctypes.byref(_params(levels=5))) <= _abi.BP_NOALLOC_SCRATCH_BYTES
