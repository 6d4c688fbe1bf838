"""Host-side checks of the C ABI: the library loads, exports every function
include/lbm.h declares, and its parameter validation works without a GPU
(no compute call is made here)."""
import ctypes

import numpy as np
import pytest

from paper_1405_2232_amd import inputs, lbm


def test_library_exports_every_declared_symbol():
    names = lbm.header_functions()
    assert len(names) >= 31
    L = ctypes.CDLL(lbm.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_library_exports_every_network_symbol():
    import os
    names = lbm.header_functions(os.path.join(os.path.dirname(lbm.HEADER), "lbmnn.h"))
    assert len(names) == 16, names
    L = ctypes.CDLL(lbm.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_network_argument_checks_without_gpu():
    """Bad sizes and alignments are rejected before any launch."""
    from paper_1405_2232_amd import nn
    L = nn.lib()
    # channel counts not multiples of 16, odd pooling sizes, bad strides
    assert L.lbmnn_conv3x3(8, 16, 0, None, 0, 0, 8, None, 8, 16, 0, 1, 4, 4, 12, 16, 1, 1, None) == -1
    assert L.lbmnn_conv3x3(8, 16, 0, None, 0, 0, 8, None, 8, 16, 8, 1, 4, 4, 16, 16, 1, 1, None) == -1
    assert L.lbmnn_conv3x3(8, 16, 0, None, 0, 0, 8, None, 8, 16, 0, 1, 4, 4, 16, 144, 1, 1, None) == -1
    assert L.lbmnn_conv3x3_wgrad(8, 128, 0, 8, 128, 0, None, 0, 0, 8, None, 8, 1, 4, 4, 128, 128, 1, None) == -1
    assert L.lbmnn_pool2(8, 16, 0, 8, 16, 0, 1, 5, 4, 16, None) == -1
    assert L.lbmnn_conv3x3(4, 16, 0, None, 0, 0, 8, None, 8, 16, 0, 1, 4, 4, 16, 16, 1, 1, None) == -1
    assert L.lbmnn_head(8, 32, 0, 8, 8, 8, 8, 1, 4, 4, 24, None) == -1
    assert L.lbmnn_adam(8, 8, 8, 8, 8, 10, 1e-3, 0.9, 0.999, 1e-8, 0, None) == -1
    assert L.lbmnn_wgrad_partials(1, 4, 4, 16, 16) > 0


def test_header_and_binding_struct_agree():
    """The ctypes mirror has one field per lbm_params member, in order."""
    import re
    txt = re.sub(r"/\*.*?\*/", "", open(lbm.HEADER).read(), flags=re.S)
    body = txt[txt.index("typedef struct {") + len("typedef struct {"):txt.index("} lbm_params;")]
    decl = []
    for stmt in body.split(";"):
        stmt = stmt.strip()
        if not stmt:
            continue
        typ, rest = stmt.split(None, 1)
        decl += [(typ, n.strip()) for n in rest.split(",")]
    fields = lbm.Params._fields_
    assert [n for n, _ in fields] == [n for _, n in decl]
    for (name, ct), (typ, _) in zip(fields, decl):
        assert (ct is ctypes.c_int) == (typ == "int"), name
        assert (ct is ctypes.c_double) == (typ == "double"), name


def _bytes(cfg, **kw):
    p = lbm.make_params(cfg, **kw)
    n = ctypes.c_size_t()
    rc = lbm.lib().lbm_workspace_bytes(ctypes.byref(p), ctypes.byref(n))
    return rc, n.value


def test_workspace_bytes_scale_with_precision():
    p, _, _ = inputs.static_droplet()
    rc64, b64 = _bytes(p, precision="fp64")
    rc32, b32 = _bytes(p, precision="fp32dev", rho_ref=0.1, T_ref=0.08)
    assert rc64 == 0 and rc32 == 0
    # two buffers of 18 planes dominate: 2*18*64*64*8 bytes for FP64
    assert b64 >= 2 * 18 * 64 * 64 * 8
    assert b32 >= 2 * 18 * 64 * 64 * 4
    assert b32 < b64


@pytest.mark.parametrize("bad", [
    dict(tau_f=0.5), dict(tau_g=0.4), dict(nx=0), dict(ny=-3), dict(cv=0.0),
    dict(eos="cs", psi_policy=3), dict(tau_f=float("nan")),
])
def test_parameter_validation(bad):
    p, _, _ = inputs.static_droplet()
    p.update(bad)
    rc, _ = _bytes(p)
    assert rc == lbm.EINVAL


def test_create_rejects_small_or_misaligned_workspace():
    p, _, _ = inputs.static_droplet()
    rc, need = _bytes(p)
    assert rc == 0
    P = lbm.make_params(p)
    h = ctypes.c_void_p()
    L = lbm.lib()
    # nothing is dereferenced: creation only carves the workspace
    fake = ctypes.c_void_p(1 << 40)
    assert L.lbm_create(ctypes.byref(P), fake, need - 256, None, ctypes.byref(h)) == lbm.ENOMEM
    assert L.lbm_create(ctypes.byref(P), ctypes.c_void_p((1 << 40) + 8), need, None,
                        ctypes.byref(h)) == lbm.EINVAL
    assert L.lbm_create(ctypes.byref(P), fake, need, None, ctypes.byref(h)) == lbm.OK
    # out-of-order and bad-argument calls fail before touching the device
    assert L.lbm_step(h, 1, lbm.PLAIN) == lbm.ESTATE
    assert L.lbm_step(h, 0, lbm.PLAIN) == lbm.EINVAL
    assert L.lbm_step(h, 1, 7) == lbm.EINVAL
    # both starts validate the host fields before any copy
    n = p["nx"] * p["ny"]
    good = np.full(n, 0.1)
    bad = good.copy()
    bad[n // 2] = 0.0
    for fn in (L.lbm_init_fields, L.lbm_init_fields_physical):
        assert fn(None, lbm._dp(good), None, None, lbm._dp(good)) == lbm.EINVAL
        assert fn(h, None, None, None, lbm._dp(good)) == lbm.EINVAL
        assert fn(h, lbm._dp(bad), None, None, lbm._dp(good)) == lbm.EINVAL
        nan_u = good.copy()
        nan_u[3] = np.nan
        assert fn(h, lbm._dp(good), lbm._dp(nan_u), None, lbm._dp(good)) == lbm.EINVAL
    assert L.lbm_batch_init_fields_physical(None, 0, lbm._dp(good), None, None,
                                            lbm._dp(good)) == lbm.EINVAL
    assert L.lbm_set_tiling(h, 96, 4) == lbm.EINVAL
    assert L.lbm_set_tiling(h, 128, 0) == lbm.EINVAL
    assert L.lbm_set_tiling(h, 128, 5) == lbm.OK
    bx, rows = ctypes.c_int(), ctypes.c_int()
    assert L.lbm_get_tiling(h, ctypes.byref(bx), ctypes.byref(rows)) == lbm.OK
    assert (bx.value, rows.value) == (128, 5)
    assert L.lbm_destroy(h) == lbm.OK


def test_strerror_names_every_status():
    L = lbm.lib()
    seen = set()
    for s in (lbm.OK, lbm.EINVAL, lbm.ENOMEM, lbm.EDEVICE, lbm.ENONFINITE, lbm.EDOMAIN, lbm.ESTATE):
        msg = L.lbm_strerror(s).decode()
        assert msg and msg != "unknown status"
        seen.add(msg)
    assert len(seen) == 7


def _host_handle(cfg, precision):
    """A handle whose workspace pointer is never dereferenced on the host:
    lbm_create only records offsets, so the pairing choice can be checked
    without a GPU (nothing here launches or copies)."""
    p = lbm.make_params(cfg, precision, 0.1, 0.08)
    L = lbm.lib()
    n = ctypes.c_size_t()
    assert L.lbm_workspace_bytes(ctypes.byref(p), ctypes.byref(n)) == 0
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(1 << 40)  # 256-byte aligned, never touched
    assert L.lbm_create(ctypes.byref(p), fake, n.value, None, ctypes.byref(h)) == 0
    return L, h


@pytest.mark.parametrize("nx,ny,precision,rows", [
    (2048, 2048, "fp32local", 35), (4096, 4096, "fp32local", 137), (1024, 1024, "fp32local", 10),
    (64, 64, "fp32local", 6), (300, 70, "fp32local", 6), (2048, 2048, "fp64", 69)])
def test_two_step_band_height_without_gpu(nx, ny, precision, rows, monkeypatch):
    """The two-step band height the launch-round model picks (128-lane
    blocks, four per CU for FP32 storage and two for FP64, 256 CUs when no
    device answers): the fewest bands minimising rounds x (2 r + 4)."""
    monkeypatch.delenv("LBM_PAIR_ROWS", raising=False)
    monkeypatch.delenv("LBM_PAIR_BX", raising=False)
    cfg = dict(inputs.static_droplet(nx=32, ny=32, radius=8, seed=1)[0], nx=nx, ny=ny)
    L, h = _host_handle(cfg, precision)
    try:
        a, r = ctypes.c_int(), ctypes.c_int()
        assert L.lbm_get_step_pairing(h, ctypes.byref(a), ctypes.byref(r)) == 0
        # on by default only where the lattice fills the device
        assert a.value == (1 if nx * ny >= 1024 * 1024 else 0) and r.value == rows
        assert L.lbm_set_step_pairing(h, 1, 0) == 0
        # an explicit height: bands of at most that many rows
        assert L.lbm_set_step_pairing(h, 1, 5) == 0
        assert L.lbm_get_step_pairing(h, ctypes.byref(a), ctypes.byref(r)) == 0
        assert r.value <= 5
        assert L.lbm_set_step_pairing(h, 1, -1) == -1
        assert L.lbm_set_step_pairing(h, 0, 0) == 0
        assert L.lbm_get_step_pairing(h, ctypes.byref(a), ctypes.byref(r)) == 0
        assert a.value == 0
    finally:
        L.lbm_destroy(h)


@pytest.mark.parametrize("precision,extra,want", [
    ("fp32local", {}, 1), ("fp32dev", {}, 1), ("fp64", {}, 1),
    ("fp32local", {"wall_x": True}, 0), ("fp32local", {"wall_x": "open", "u_in": 0.01}, 0),
    ("fp32local", {"beta": 0.5}, 1), ("fp32local", {"G": 0.0, "beta": 0.5}, 1),
    ("fp32local", {"wall_y": True}, 1)])
def test_two_step_eligibility_without_gpu(precision, extra, want):
    cfg = dict(inputs.static_droplet(nx=40, ny=30, radius=8, seed=1)[0], **extra)
    L, h = _host_handle(cfg, precision)
    try:
        a, r = ctypes.c_int(), ctypes.c_int()
        assert L.lbm_set_step_pairing(h, 1, 0) == 0  # a small lattice: off by default
        assert L.lbm_get_step_pairing(h, ctypes.byref(a), ctypes.byref(r)) == 0
        assert a.value == want
    finally:
        L.lbm_destroy(h)


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asked for more it says so and exits with
    status 2 before touching a device."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_checkpoint_load_rejects_other_files_before_any_copy(tmp_path):
    """lbm_load checks the file's header against the handle before it
    touches the device: a file of another format, of another lattice size
    or cut short is LBM_EINVAL (with no device here, a copy would have
    failed with LBM_EDEVICE instead)."""
    import struct
    cfg = inputs.static_droplet(nx=32, ny=32, radius=8, seed=1)[0]
    L, h = _host_handle(cfg, "fp32local")
    try:
        def header(magic=b"LBMCKPT2", nx=32, ny=32):
            # magic, nx, ny, precision, cur, steps, clamps, bytes, plane, pitch, rpitch, rho_ref, cvT_ref
            return struct.pack("<8s4iqQQqii2d", magic, nx, ny, 2, 0, 0, 0, 0, 0, 0, 0, 0.1, 0.08)
        cases = {"other format": header(magic=b"LBMCKPT1") + b"\0" * 64,
                 "other size": header(nx=64) + b"\0" * 64,
                 "short header": header()[:20],
                 "empty": b""}
        for name, data in cases.items():
            path = tmp_path / (name.replace(" ", "_") + ".ckpt")
            path.write_bytes(data)
            assert L.lbm_load(h, str(path).encode()) == lbm.EINVAL, name
        assert L.lbm_load(h, str(tmp_path / "missing.ckpt").encode()) == lbm.EINVAL
    finally:
        L.lbm_destroy(h)
