"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/geomst.h declares, and rejects bad arguments before
touching the device."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from paper_2104_01126_amd import geomst as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(G.LIB_PATH):
        from paper_2104_01126_amd import build
        build.build()
    return G.load()


def test_exports_every_declared_symbol(lib):
    declared = G.declared_symbols()
    assert "geomst_emst" in declared and "geomst_hdbscan_dev" in declared
    out = subprocess.run(["nm", "-D", "--defined-only", G.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    for name in declared:
        assert name in exported, name
        assert hasattr(lib, name)


def test_header_compiles_as_c():
    src = "#include \"geomst.h\"\nint main(void){ geomst_stats_t s; (void)s; int (*f)(void) = geomst_version; return f != 0 ? 0 : 1; }\n"
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), "-x", "c",
                        "-", "-fsyntax-only"], input=src, text=True, capture_output=True)
    assert r.returncode == 0, r.stderr


def test_version(lib):
    assert G.version() == 100


def _emst_rc(lib, pts, n, d, edges):
    return lib.geomst_emst(pts, n, d, edges, None)


def test_rejects_bad_arguments_without_device(lib):
    p = np.zeros((4, 3))
    e = np.zeros((3, 2), np.int64)
    assert _emst_rc(lib, None, 4, 3, e.ctypes.data) == G.EINVAL
    assert _emst_rc(lib, p.ctypes.data, 0, 3, e.ctypes.data) == G.EINVAL
    assert _emst_rc(lib, p.ctypes.data, 4, 0, e.ctypes.data) == G.EINVAL
    assert _emst_rc(lib, p.ctypes.data, 4, 8, e.ctypes.data) == G.EINVAL
    assert _emst_rc(lib, p.ctypes.data, 4, 3, None) == G.EINVAL
    assert _emst_rc(lib, p.ctypes.data, (1 << 26) + 1, 3, e.ctypes.data) == G.EINVAL
    assert "n must be" in G.last_error()
    cd = np.zeros(4)
    assert lib.geomst_hdbscan(p.ctypes.data, 4, 3, 0, cd.ctypes.data, e.ctypes.data, None) == G.EINVAL
    assert lib.geomst_hdbscan(p.ctypes.data, 4, 3, 5, cd.ctypes.data, e.ctypes.data, None) == G.EINVAL
    assert lib.geomst_hdbscan(p.ctypes.data, 4, 3, 65, cd.ctypes.data, e.ctypes.data, None) == G.EINVAL
    assert lib.geomst_emst_dev(None, 4, 3, None, None, None, None) == G.EINVAL
    assert lib.geomst_emst_dev_noalloc(None, 4, 3, None, None, None, None) == G.EINVAL
    # approximate OPTICS: rho and minPts are checked before any device call
    for mp, rho in ((0, 0.5), (65, 0.5), (3, 0.0), (3, -1.0), (3, float("nan")), (3, float("inf")), (5, 0.5)):
        assert lib.geomst_optics_approx(p.ctypes.data, 4, 3, mp, rho, cd.ctypes.data, e.ctypes.data,
                                        None) == G.EINVAL, (mp, rho)
    assert lib.geomst_optics_approx_dev(None, 4, 3, 3, 0.5, None, None, None, None, None, None) == G.EINVAL
    o = np.zeros(4, np.int64)
    r = np.zeros(4)
    w = np.zeros(3)
    assert lib.geomst_dendrogram(e.ctypes.data, w.ctypes.data, 4, 4, None, None, o.ctypes.data,
                                 r.ctypes.data) == G.EINVAL   # start out of range
    assert lib.geomst_dendrogram(e.ctypes.data, w.ctypes.data, 0, 0, None, None, o.ctypes.data,
                                 r.ctypes.data) == G.EINVAL   # n < 1
    assert lib.geomst_dendrogram(None, w.ctypes.data, 4, 0, None, None, o.ctypes.data,
                                 r.ctypes.data) == G.EINVAL   # edges NULL
    assert lib.geomst_dendrogram_dev(e.ctypes.data, w.ctypes.data, 4, 0, None, None, None, None,
                                     None) == G.EINVAL          # order NULL
    nmax = G.header_constant("GEOMST_NOALLOC_MAX_POINTS")
    assert lib.geomst_emst_dev_noalloc(p.ctypes.data, nmax + 1, 3, e.ctypes.data, None, None, None) == G.EINVAL
    assert "GEOMST_NOALLOC_MAX_POINTS" in G.last_error()
    with pytest.raises(G.GeomstError):
        G.emst(np.zeros((4, 9)))


def test_options(lib):
    assert lib.geomst_set_option(b"beta_growth", 1.0) == G.EINVAL
    assert lib.geomst_set_option(b"beta_growth", float("nan")) == G.EINVAL
    assert lib.geomst_set_option(b"no_such_option", 2.0) == G.EINVAL
    assert lib.geomst_set_option(b"beta_growth", 2.0) == G.OK
    assert lib.geomst_set_option(b"beta_growth", 0.0) == G.OK
    assert lib.geomst_set_option(b"list_capacity_scale", 0.0) == G.EINVAL
    assert lib.geomst_set_option(b"kernel_timing", 2.0) == G.EINVAL
    assert lib.geomst_set_option(b"beta_start_quantile", 1.5) == G.EINVAL
    assert lib.geomst_set_option(b"beta_start_quantile", -0.1) == G.EINVAL
    assert lib.geomst_set_option(b"beta_start_quantile", 1.0 / 64) == G.OK
    assert lib.geomst_set_option(b"beta_start_quantile", 0.0) == G.OK  # back to the default
    assert lib.geomst_set_option(b"schedule", 4.0) == G.EINVAL
    assert lib.geomst_set_option(b"schedule", 0.0) == G.OK
    assert lib.geomst_set_option(b"separation_mode", 2.0) == G.EINVAL
    assert lib.geomst_set_option(b"separation_mode", 0.0) == G.OK
    assert lib.geomst_set_option(b"server_share_scale", 0.0) == G.EINVAL
    assert lib.geomst_set_option(b"beta_schedule", 2.0) == G.EINVAL
    assert lib.geomst_set_option(b"beta_schedule", 1.0) == G.OK
    assert lib.geomst_set_option(b"beta_schedule", 0.0) == G.OK


def _c_layout(exprs):
    """Evaluate size_t expressions over include/geomst.h with gcc."""
    body = " ".join(f'printf("%zu ", (size_t)({e}));' for e in exprs)
    src = ("#include <stdio.h>\n#include <stddef.h>\n#include \"geomst.h\"\n"
           f"int main(void){{ {body} return 0; }}\n")
    exe = os.path.join(ROOT, "_build_stats_probe")
    try:
        subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), "-x", "c", "-", "-o", exe],
                       input=src, text=True, check=True)
        return list(map(int, subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()))
    finally:
        if os.path.exists(exe):
            os.remove(exe)


def test_stats_struct_layout(lib):
    s = G.stats()
    assert isinstance(s.rounds, int)
    # the ctypes mirror has the size of the C struct
    size, off = _c_layout(["sizeof(geomst_stats_t)", "offsetof(geomst_stats_t, kernel_ms)"])
    assert ctypes.sizeof(G._Stats) == size
    assert G._Stats.kernel_ms.offset == off


def test_server_struct_layouts():
    structs = [("geomst_server_cfg_t", G.ServerCfg), ("geomst_request_info_t", G.RequestInfo),
               ("geomst_server_stats_t", G.ServerStats), ("geomst_instance_t", G.Instance),
               ("geomst_batch_item_t", G.BatchItem)]
    exprs = []
    for cname, py in structs:
        exprs.append(f"sizeof({cname})")
        exprs += [f"offsetof({cname}, {f})" for f, _ in py._fields_]
    vals = iter(_c_layout(exprs))
    for cname, py in structs:
        assert next(vals) == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert next(vals) == getattr(py, f).offset, (cname, f)


def test_server_validation_without_device(lib):
    h = ctypes.c_void_p()
    bad = [G.ServerCfg(0, 17, -1, 0, 0, 0), G.ServerCfg(0, 2, -1, 0, -1, 0), G.ServerCfg(0, 2, -1, 0, 0, (1 << 26) + 1),
           G.ServerCfg(0, 2, -2, 0, 0, 0), G.ServerCfg(0, -1, -1, 0, 0, 0)]
    for cfg in bad:
        assert lib.geomst_server_create(ctypes.byref(cfg), ctypes.byref(h)) == G.EINVAL
        assert not h.value
    assert lib.geomst_server_create(None, None) == G.EINVAL
    t = ctypes.c_uint64()
    req = G.Instance()
    assert lib.geomst_submit(None, ctypes.byref(req), ctypes.byref(t)) == G.EINVAL
    assert lib.geomst_wait(None, 1, 0, None) == G.EINVAL
    assert lib.geomst_cancel(None, 1) == G.EINVAL
    assert lib.geomst_server_stats(None, None) == G.EINVAL
    lib.geomst_server_destroy(None)  # no-op


def test_batch_validation_without_device(lib):
    items = (G.BatchItem * 2)()
    items[0].offset, items[0].n, items[0].d, items[0].min_pts = 0, 5, 2, 0
    items[1].offset, items[1].n, items[1].d, items[1].min_pts = 6, 5, 2, 0   # not packed
    p = np.zeros((11, 2))
    assert lib.geomst_batch_dev(p.ctypes.data, 2, items, 2, p.ctypes.data, None, None, None, None, None) == G.EINVAL
    assert "batch item 1" in G.last_error()
    items[1].offset = 5
    items[1].d = 3   # d above the stride
    assert lib.geomst_batch_dev(p.ctypes.data, 2, items, 2, p.ctypes.data, None, None, None, None, None) == G.EINVAL
    items[1].d, items[1].min_pts = 2, 6   # min_pts above n
    assert lib.geomst_batch_dev(p.ctypes.data, 2, items, 2, p.ctypes.data, None, None, None, None, None) == G.EINVAL
    assert lib.geomst_batch_dev(p.ctypes.data, 8, items, 2, p.ctypes.data, None, None, None, None, None) == G.EINVAL
    inst = (G.Instance * 1)()
    x = np.array([[0.0, np.inf], [1.0, 1.0]])
    e = np.zeros((1, 2), np.int64)
    inst[0].points, inst[0].n, inst[0].d, inst[0].min_pts, inst[0].edges = x.ctypes.data, 2, 2, 0, e.ctypes.data
    assert lib.geomst_batch(inst, 1) == G.EDOM and inst[0].status == G.EDOM


def test_pack_layout():
    a = np.arange(6.0).reshape(3, 2)
    b = np.arange(9.0).reshape(3, 3) + 100
    arena, items, stride = G.pack([a, b], [0, 2])
    assert stride == 3 and arena.shape == (6, 3)
    assert np.array_equal(arena[:3, :2], a) and np.all(arena[:3, 2] == 0.0) and np.array_equal(arena[3:], b)
    assert (items[1].offset, items[1].n, items[1].d, items[1].min_pts) == (3, 3, 3, 2)


def test_tuning_cache_parsing(lib, tmp_path):
    """The tuning cache loader (host only): a valid file loads, a malformed
    or out-of-range line is rejected and leaves the table unchanged, a
    missing file is ENOENT, NULL clears the table."""
    good = tmp_path / "tune.jsonl"
    good.write_text('# tuner output\n'
                    '{"kind": "emst", "d": 3, "nlog2": 25, "bccp_chunk": 1024, "small_level_switch": 1024, '
                    '"small_level_max": 2048, "beta_growth": 3.0, "ms": 170.2}\n'
                    '\n'
                    '{"kind": "hdbscan", "d": 5, "nlog2": 21, "refresh_divisor": 512, "beta_start_quantile": 0.0}\n')
    assert lib.geomst_load_tuning(str(good).encode()) == G.OK
    for bad in ['{"kind": "emst", "d": 3}',                                        # no nlog2
                '{"kind": "kmeans", "d": 3, "nlog2": 10}',                         # bad kind
                '{"kind": "emst", "d": 3, "nlog2": 10, "bccp_chunk": 100}',        # not a multiple of 64
                '{"kind": "emst", "d": 9, "nlog2": 10}',                           # d out of range
                '{"kind": "emst", "d": 3, "nlog2": 10, "beta_growth": 1.0}',       # growth must exceed 1
                '"kind": "emst"']:                                                 # not an object
        p = tmp_path / "bad.jsonl"
        p.write_text(bad + "\n")
        assert lib.geomst_load_tuning(str(p).encode()) == G.EINVAL, bad
        assert "line 1" in G.last_error()
    assert lib.geomst_load_tuning(str(tmp_path / "missing.jsonl").encode()) == G.ENOENT
    assert lib.geomst_load_tuning(None) == G.OK


def test_error_codes_match_header():
    """The binding's status constants are the header's values."""
    from paper_2104_01126_amd import geomst as G
    for name in ("OK", "EINVAL", "EDOM", "ENOMEM", "EDEVICE", "EBUSY", "ETIMEDOUT", "ECANCELED", "EINTERNAL",
                 "ENOENT"):
        assert getattr(G, name) == G.header_constant("GEOMST_" + name), name
    vals = [G.header_constant("GEOMST_" + n) for n in ("EINVAL", "EDOM", "ENOMEM", "EDEVICE", "EBUSY", "ETIMEDOUT",
                                                       "ECANCELED", "EINTERNAL", "ENOENT")]
    assert len(set(vals)) == len(vals) and all(v < 0 for v in vals)
