"""C ABI without a GPU: the library loads, exports every declared function,
and rejects bad arguments before any HIP call."""
import ctypes
import os
import re

import pytest

from paper_2310_02926_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "binning.h")

F = 0x10000  # fake, suitably aligned device addresses: never dereferenced here


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b((?:bin|binsrv)_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    L = B.lib()
    names = declared_functions()
    assert len(names) >= 20
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(B.EXPORTS)


def test_status_strings_and_version():
    assert B.status_string(B.BIN_OK) == "BIN_OK"
    assert B.status_string(B.BIN_ERR_INVALID_ARG) == "BIN_ERR_INVALID_ARG"
    assert B.status_string(-99) == "BIN_ERR_UNKNOWN"
    assert re.match(r"\d+\.\d+\.\d+", B.bin_version())


def good(**over):
    args = dict(coords=[F, F + 0x100, F + 0x200], attrs=[F + 0x300, F + 0x400], n=1000, axes=(0, 1),
                bounds=(0.0, 1.0, 0.0, 1.0), nx=16, ny=8, ops=B.OPS_ALL,
                out={"count": F + 0x500, "sum": [F + 0x600, F + 0x700], "min": [F + 0x800, F + 0x900],
                     "max": [F + 0xA00, F + 0xB00], "avg": [F + 0xC00, F + 0xD00]},
                coord_dtype=B.BIN_F32, attr_dtype=B.BIN_F32)
    args.update(over)
    return args


def validate(**over):
    return B.bin_validate(**good(**over))


def test_valid_request_passes():
    assert validate() == B.BIN_OK
    assert validate(n=0) == B.BIN_OK
    assert validate(n=0xFFFFFFFF) == B.BIN_OK
    assert validate(attrs=[], ops=B.COUNT, out={"count": F}) == B.BIN_OK
    assert validate(bounds=None) == B.BIN_OK  # bounds on the fly


@pytest.mark.parametrize("over,frag", [
    (dict(n=-1), "n ="),
    (dict(n=0x100000000), "n ="),
    (dict(nx=0), "nx, ny"),
    (dict(ny=-3), "nx, ny"),
    (dict(nx=65536, ny=65536), "exceeds"),
    (dict(axes=(0, 3)), "axes[1]"),
    (dict(axes=(-1, 0)), "axes[0]"),
    (dict(bounds=(0.0, float("nan"), 0.0, 1.0)), "finite"),
    (dict(bounds=(0.0, float("inf"), 0.0, 1.0)), "finite"),
    (dict(bounds=(1.0, 1.0, 0.0, 1.0)), "lo < hi"),
    (dict(bounds=(0.0, 1.0, 2.0, 1.0)), "lo < hi"),
    (dict(bounds=(-1.7e308, 1.7e308, 0.0, 1.0)), "overflows"),
    (dict(bounds=(0.0, 1e-320, 0.0, 1.0)), "scale"),
    (dict(ops=0), "no reduction"),
    (dict(ops=0x4000), "unknown bits"),
    (dict(ops=B.OPS_ALL | B.PREC_PLAIN | B.PREC_F64), "exclusive"),
    (dict(attrs=[], ops=B.SUM), "no attribute"),
    (dict(coord_dtype=7), "dtype"),
    (dict(attr_dtype=5), "dtype"),
    (dict(coords=[F + 2, F, F]), "misaligned"),
    (dict(coords=[0, F, F]), "NULL"),
    (dict(attrs=[F, 0]), "NULL"),
    (dict(out={"sum": [F, F]}), "count"),
    (dict(out={"count": F, "sum": [F, F], "min": [F, F], "max": [F, F]}), "avg"),
    (dict(out={"count": F, "sum": [F, 0], "min": [F, F], "max": [F, F], "avg": [F, F]}), "sum[1]"),
    (dict(out={"count": F, "sum": [F + 4, F], "min": [F, F], "max": [F, F], "avg": [F, F]}), "misaligned"),
    (dict(attrs=[F] * 17), "attrs->ncols"),
])
def test_invalid_arguments_rejected(over, frag):
    assert validate(**over) == B.BIN_ERR_INVALID_ARG
    assert frag in B.last_error(), B.last_error()


def test_bin_particles_rejects_before_any_hip_call():
    # No GPU in this process: an argument error must come back without the
    # library ever reaching the HIP runtime.
    with pytest.raises(B.BinError) as ei:
        B.bin_particles(**good(nx=0), stream=0)
    assert ei.value.status == B.BIN_ERR_INVALID_ARG
    with pytest.raises(B.BinError) as ei:
        B.bin_particles(**good(bounds=(0.0, 0.0, 0.0, 1.0)), stream=0)
    assert ei.value.status == B.BIN_ERR_INVALID_ARG
    # the allocation-free variant runs the same checks first
    for over in (dict(nx=0), dict(bounds=(0.0, 0.0, 0.0, 1.0)), dict(ops=0)):
        with pytest.raises(B.BinError) as ei:
            B.bin_particles_noalloc(**good(**over), stream=0)
        assert ei.value.status == B.BIN_ERR_INVALID_ARG


def test_prepared_call_passes_the_same_arguments():
    # A request marshalled once (binding.Call) reaches the same checks with
    # the same arguments as bin_particles, launch after launch.
    for over, frag in ((dict(nx=0), "nx, ny"), (dict(axes=(0, 3)), "axes[1]"), (dict(ops=0), "no reduction"),
                       (dict(bounds=(0.0, 1.0, 2.0, 1.0)), "lo < hi")):
        call = B.Call(**good(**over))
        for _ in range(2):
            with pytest.raises(B.BinError) as ei:
                call.launch(stream=0)
            assert ei.value.status == B.BIN_ERR_INVALID_ARG and frag in B.last_error(), B.last_error()


def test_plain_sum_outputs_may_be_4_byte_aligned():
    out = {"count": F, "sum": [F + 4, F], "min": [F, F], "max": [F, F], "avg": [F + 4, F]}
    assert validate(out=out, ops=B.OPS_ALL | B.PREC_PLAIN) == B.BIN_OK
    assert validate(out=out) == B.BIN_ERR_INVALID_ARG  # default: double outputs


def test_f64_attributes_need_8_byte_min_max():
    out = {"count": F, "sum": [F, F], "min": [F + 4, F], "max": [F, F], "avg": [F, F]}
    assert validate(out=out, attr_dtype=B.BIN_F64) == B.BIN_ERR_INVALID_ARG
    assert validate(out=out, attr_dtype=B.BIN_F32) == B.BIN_OK


def test_single_hip_runtime_mapped():
    import torch  # noqa: F401
    B.lib()
    maps = open("/proc/self/maps").read()
    libs = {l.split()[-1] for l in maps.splitlines() if "libamdhip64" in l}
    assert len(libs) == 1, libs


def test_multi_grid_rejects_bad_specs_before_any_hip_call():
    a = good()
    grid = dict(axes=(0, 2), bounds=(0.0, 1.0, 0.0, 1.0), nx=16, ny=8, ops=B.OPS_ALL, out=a["out"])
    bad = dict(grid, nx=0)
    with pytest.raises(B.BinError) as ei:
        B.bin_particles_multi(a["coords"], a["attrs"], 1000, [grid, bad], stream=0, coord_dtype=B.BIN_F32,
                              attr_dtype=B.BIN_F32)
    assert ei.value.status == B.BIN_ERR_INVALID_ARG
    assert "request 1" in B.last_error(), B.last_error()
    with pytest.raises(B.BinError) as ei:
        B.bin_particles_multi(a["coords"], a["attrs"], 1000, [dict(grid, axes=(0, 3))], stream=0,
                              coord_dtype=B.BIN_F32, attr_dtype=B.BIN_F32)
    assert ei.value.status == B.BIN_ERR_INVALID_ARG
    L = B.lib()
    assert L.bin_particles_multi(None, None, 0, None, 0, None) == B.BIN_ERR_INVALID_ARG
    c, keep = B.columns([F, F + 0x100], B.BIN_F32)
    assert L.bin_particles_multi(ctypes.byref(c), None, 10, None, 2, None) == B.BIN_ERR_INVALID_ARG
    assert L.bin_particles_multi(ctypes.byref(c), None, 10, None, -1, None) == B.BIN_ERR_INVALID_ARG


def test_multi_grid_graph_rejects_bad_specs_before_any_hip_call():
    """bin_graph_create_multi checks its specs as bin_particles_multi does,
    and a NULL graph handle, before any HIP call (no GPU here)."""
    a = good()
    grid = dict(axes=(0, 2), bounds=(0.0, 1.0, 0.0, 1.0), nx=16, ny=8, ops=B.OPS_ALL, out=a["out"])
    with pytest.raises(B.BinError) as ei:
        B.BinGraph.multi(a["coords"], a["attrs"], 1000, [grid, dict(grid, ny=-3)], coord_dtype=B.BIN_F32,
                         attr_dtype=B.BIN_F32)
    assert ei.value.status == B.BIN_ERR_INVALID_ARG
    assert "request 1" in B.last_error(), B.last_error()
    L = B.lib()
    c, keep = B.columns([F, F + 0x100], B.BIN_F32)
    h = ctypes.c_void_p()
    assert L.bin_graph_create_multi(ctypes.byref(c), None, 10, None, 0, None) == B.BIN_ERR_INVALID_ARG
    assert L.bin_graph_create_multi(None, None, 10, None, 1, ctypes.byref(h)) == B.BIN_ERR_INVALID_ARG
    assert L.bin_graph_create_multi(ctypes.byref(c), None, 10, None, 0, ctypes.byref(h)) == B.BIN_ERR_INVALID_ARG
    assert not h.value


def test_async_rejects_before_any_hip_call():
    args = good(nx=0)
    with pytest.raises(B.BinError) as ei:
        B.bin_particles_async(**args, src_stream=0, bin_stream=0)
    assert ei.value.status == B.BIN_ERR_INVALID_ARG
    with pytest.raises(B.BinError) as ei:
        B.bin_particles_async(**good(axes=(0, 5)), src_stream=0, bin_stream=0)
    assert ei.value.status == B.BIN_ERR_INVALID_ARG


def good_nd(**over):
    a = good()
    args = dict(coords=a["coords"], attrs=a["attrs"], n=1000, axes=(0, 1, 2),
                bounds=(0.0, 1.0, 0.0, 1.0, -1.0, 1.0), dims=(16, 8, 4), ops=B.OPS_ALL, out=a["out"],
                coord_dtype=B.BIN_F32, attr_dtype=B.BIN_F32)
    args.update(over)
    return args


def test_nd_valid_requests_pass():
    assert B.bin_validate_nd(**good_nd()) == B.BIN_OK
    assert B.bin_validate_nd(**good_nd(axes=(2,), bounds=(0.0, 1.0), dims=(100,))) == B.BIN_OK
    assert B.bin_validate_nd(**good_nd(axes=(2, 0), bounds=(0.0, 1.0, 5.0, 6.0), dims=(3, 7))) == B.BIN_OK
    assert B.bin_validate_nd(**good_nd(axes=(1, 1, 1))) == B.BIN_OK
    assert B.bin_validate_nd(**good_nd(bounds=None)) == B.BIN_OK
    # f32 coordinates: the folded axes 1 and 2 must stay exact in binary32
    assert B.bin_validate_nd(**good_nd(dims=(1, 4096, 4096))) == B.BIN_OK
    assert B.bin_validate_nd(**good_nd(dims=(1, 4097, 4096), coord_dtype=B.BIN_F64)) == B.BIN_OK


@pytest.mark.parametrize("over,frag", [
    (dict(ndim=0), "ndim"),
    (dict(ndim=4, axes=(0, 1, 2, 0), dims=(2, 2, 2, 2), bounds=(0.0, 1.0) * 4), "ndim"),
    (dict(axes=(0, 1, 3)), "axes[2]"),
    (dict(axes=(0, 3, 1)), "axes[1]"),
    (dict(dims=(16, 0, 4)), "dims[1]"),
    (dict(dims=(65536, 65536, 1)), "product"),
    (dict(dims=(1, 4097, 4096)), "2^24"),
    (dict(bounds=(0.0, 1.0, 0.0, 1.0, 1.0, 1.0)), "axis 2"),
    (dict(bounds=(0.0, 1.0, float("nan"), 1.0, 0.0, 1.0)), "axis 1"),
    (dict(axes=(0,), bounds=(2.0, 1.0), dims=(4,)), "axis 0"),
    (dict(coords=[F, F + 0x100, 0]), "column 2 is NULL"),
    (dict(coords=[F, F + 0x100, F + 0x202]), "column 2 is misaligned"),
    (dict(attrs=[], ops=B.OPS_ALL, out={"count": F}), "no attribute"),
])
def test_nd_invalid_arguments_rejected(over, frag):
    assert B.bin_validate_nd(**good_nd(**over)) == B.BIN_ERR_INVALID_ARG
    assert frag in B.last_error(), B.last_error()


def test_nd_rejects_before_any_hip_call():
    with pytest.raises(B.BinError) as ei:
        B.bin_particles_nd(**good_nd(dims=(16, 8, 0)), stream=0)
    assert ei.value.status == B.BIN_ERR_INVALID_ARG
    L = B.lib()
    assert L.bin_particles_nd(None, None, 0, 3, None, None, None, 1, None, None) == B.BIN_ERR_INVALID_ARG


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the built library every entry point raises: there is no
    fallback path."""
    monkeypatch.setattr(B, "_lib", None)
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "libbinning.so"))
    with pytest.raises(RuntimeError, match="is missing"):
        B.lib()
    with pytest.raises(RuntimeError, match="is missing"):
        B.bin_version()
    with pytest.raises(RuntimeError, match="is missing"):
        B.bin_particles([0x1000, 0x2000], [0x3000], 10, (0, 1), (0.0, 1.0, 0.0, 1.0), 4, 4, B.COUNT,
                        {"count": 0x4000}, coord_dtype=B.BIN_F32, attr_dtype=B.BIN_F32)


def test_product_path_never_reaches_the_oracle():
    """The package (Python and native sources) imports, loads and calls
    nothing under oracle/, and importing it leaves the oracle unloaded."""
    import ast
    import subprocess
    import sys
    pkg = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2310_02926_amd")
    for name in os.listdir(pkg):
        if name.endswith(".py"):
            tree = ast.parse(open(os.path.join(pkg, name)).read())
            for node in ast.walk(tree):
                if isinstance(node, ast.Import):
                    assert not any(a.name.split(".")[0] == "oracle" for a in node.names), name
                elif isinstance(node, ast.ImportFrom):
                    assert (node.module or "").split(".")[0] != "oracle", name
    csrc = os.path.join(pkg, "csrc")
    for name in os.listdir(csrc):
        text = open(os.path.join(csrc, name), errors="replace").read()
        assert "oracle" not in text, name
    code = ("import sys; import paper_2310_02926_amd.binding, paper_2310_02926_amd.synth; "
            "print(any(m == 'oracle' or m.startswith('oracle.') for m in sys.modules))")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=os.path.dirname(pkg))
    assert out.returncode == 0 and out.stdout.strip() == "False", out.stderr
