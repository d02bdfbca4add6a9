"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every symbol include/fclsh.h declares, and its host-only parameter draw
(Alg. 1 + Alg. 2 random choices) agrees with the oracle's independent
implementation of the same SplitMix64 recipe."""
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
import paper_1602_02620_amd as fc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fclsh.h")


def header_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fclsh_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_binding_exports():
    assert header_symbols() == sorted(fc.EXPORTS)


def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", fc.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (fclsh_[a-z_]+)\b", out))
    missing = [s for s in header_symbols() if s not in exported]
    assert not missing, missing
    lib = fc.lib()
    for s in header_symbols():
        getattr(lib, s)


def test_exports_are_plain_c():
    # extern "C": no mangled fclsh symbols leak through
    out = subprocess.run(["nm", "-D", "--defined-only", fc.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    assert "fclsh_" in out
    mangled = [ln for ln in out.splitlines() if re.search(r"\b_Z\S*fclsh", ln)]
    assert not mangled, mangled[:3]


@pytest.mark.parametrize("d,r,seed,t", [(128, 4, 3001, 0), (256, 8, 3002, 0), (64, 6, 3003, 0),
                                        (512, 12, 3004, 0), (256, 10, 3005, 0), (1024, 20, 3006, 0),
                                        (101, 13, 7, 0), (300, 9, 8, 3), (5, 2, 9, 0), (64, 22, 10, 2)])
def test_params_match_oracle(d, r, seed, t):
    p = fc.derive_params(d, r, seed, partitions=t)
    o = oracle.derive_params(d, r, seed, override_t=t)
    assert p["t"] == o.t and p["r_part"] == o.rpart
    assert np.array_equal(p["part"], o.part)
    assert np.array_equal(p["col"], o.col)
    assert np.array_equal(p["b"], o.b)


@pytest.mark.parametrize("d,r,seed,times", [(128, 2, 3011, 4), (128, 3, 3012, 3), (64, 5, 3013, 2),
                                            (100, 2, 3014, 3), (7, 1, 3015, 2)])
def test_replicated_params_match_oracle(d, r, seed, times):
    # Alg. 1's replication: the draws of times*d coordinates at radius times*r, one part
    p = fc.derive_params(d, r, seed, replicate=times)
    o = oracle.derive_params(times * d, times * r, seed, override_t=1)
    assert p["t"] == 1 and p["r_part"] == o.rpart == times * r
    assert np.array_equal(p["part"], o.part)
    assert np.array_equal(p["col"], o.col)
    assert np.array_equal(p["b"], o.b)


def test_preprocessing_matches_oracle():
    for n in [2, 3, 1000, 10000, 65536, 1 << 20, 10 ** 7, 1 << 40]:
        for c in [1.01, 1.1, 1.5, 2.0, 2.5, 3.0, 7.0]:
            for r in range(1, 65):
                got = fc.preprocessing(n, r, c)
                assert (got["replicate"], got["partitions"]) == oracle.preprocessing(n, r, c), (n, r, c)


@pytest.mark.parametrize("n,r,c", [(1, 3, 2.0), (1000, 0, 2.0), (1000, 3, 1.0), (1000, 3, float("nan"))])
def test_preprocessing_errors(n, r, c):
    with pytest.raises(fc.FclshError) as e:
        fc.preprocessing(n, r, c)
    assert e.value.status == fc.FCLSH_EINVAL


@pytest.mark.parametrize("d,r,t,times", [(64, 4, 0, 0), (31, 4, 0, 0), (32, 4, 0, 0), (100, 6, 0, 0),
                                         (128, 10, 0, 0), (96, 12, 3, 0), (40, 2, 0, 2)])
def test_exclude_column0_params_match_oracle(d, r, t, times):
    # the Sec. 3.3 variant: library and oracle draw the same columns from 1..D-1
    p = fc.derive_params(d, r, 77, partitions=t, replicate=times, exclude_column0=True)
    k = max(1, times)
    o = oracle.derive_params(k * d, k * r, 77, override_t=t if times == 0 else 1, exclude_column0=True)
    assert p["t"] == o.t and p["r_part"] == o.rpart
    assert np.array_equal(p["part"], o.part)
    assert np.array_equal(p["col"], o.col) and p["col"].min() >= 1
    assert np.array_equal(p["b"], o.b)
    # without the option the draws differ (column 0 is a legal target there)
    q = fc.derive_params(d, r, 77, partitions=t, replicate=times)
    assert not np.array_equal(q["col"], p["col"])


@pytest.mark.parametrize("d,r,t,times,status", [(64, 2, 2, 3, fc.FCLSH_EINVAL),        # with partitions
                                                (2048, 1, 0, 3, fc.FCLSH_EUNSUPPORTED),  # 6144 coordinates
                                                (64, 4, 0, 3, fc.FCLSH_EUNSUPPORTED),    # radius 12: 2^13 columns
                                                (64, 2, 0, -1, fc.FCLSH_EINVAL)])
def test_replication_errors(d, r, t, times, status):
    with pytest.raises(fc.FclshError) as e:
        fc.derive_params(d, r, 1, partitions=t, replicate=times)
    assert e.value.status == status


@pytest.mark.parametrize("d,r,t,status", [(0, 3, 0, fc.FCLSH_EINVAL), (10, -1, 0, fc.FCLSH_EINVAL),
                                          (64, 24, 0, fc.FCLSH_EUNSUPPORTED),  # r' = 12: 2^13 columns
                                          (4, 2, 5, fc.FCLSH_EUNSUPPORTED),    # more parts than coordinates
                                          (600_000, 2, 0, fc.FCLSH_EUNSUPPORTED)])  # above 2^19
def test_param_errors(d, r, t, status):
    with pytest.raises(fc.FclshError) as e:
        fc.derive_params(d, r, 1, partitions=t)
    assert e.value.status == status
    assert fc.lib().fclsh_last_error().decode()


def test_largest_supported_family():
    p = fc.derive_params(64, 11, 1, partitions=1)  # r' = 11: D = 4096 columns
    assert p["r_part"] == 11 and int(p["col"].max()) < 4096


def _derive_with(opts):
    d = 300
    part = np.zeros(d, np.int32)
    col = np.zeros(d, np.int32)
    b = np.zeros(d, np.uint64)
    t, rp = fc.ctypes.c_int32(), fc.ctypes.c_int32()
    st = fc.lib().fclsh_derive_params(d, 9, 8, fc.ctypes.byref(opts), fc.ctypes.byref(t), fc.ctypes.byref(rp),
                                      part.ctypes.data, col.ctypes.data, b.ctypes.data)
    return st, t.value


def test_build_opts_struct_size():
    # a full struct reads every field: partitions = 3 takes effect
    st, t = _derive_with(fc.BuildOpts.make(partitions=3))
    assert st == fc.FCLSH_OK and t == 3
    # a caller built against a struct that ends before `partitions` gets the
    # default for it (t = 1 at r = 9), whatever lies past its size
    o = fc.BuildOpts.make(partitions=3)
    o.struct_size = 4
    st, t = _derive_with(o)
    assert st == fc.FCLSH_OK and t == 1
    # size 0 or larger than the library's struct is refused
    for bad in (0, fc.ctypes.sizeof(fc.BuildOpts) + 8):
        o = fc.BuildOpts.make()
        o.struct_size = bad
        st, _ = _derive_with(o)
        assert st == fc.FCLSH_EINVAL
    o = fc.BuildOpts.make()
    o.test_flags = 2  # bit 0 is the only test flag
    assert _derive_with(o)[0] == fc.FCLSH_EINVAL
    o.test_flags = 1
    assert _derive_with(o)[0] == fc.FCLSH_OK


def test_header_struct_layout_matches_binding():
    # the C compiler's layout of fclsh_build_opts equals the binding's
    src = ("#include <stddef.h>\n#include <stdio.h>\n#include \"fclsh.h\"\n"
           "int main(void){printf(\"%zu\", sizeof(fclsh_build_opts));"
           + "".join(f"printf(\" %zu\", offsetof(fclsh_build_opts, {f}));" for f, _ in fc.BuildOpts._fields_)
           + "return 0;}\n")
    import tempfile
    with tempfile.TemporaryDirectory() as tmp:
        c = os.path.join(tmp, "layout.c")
        exe = os.path.join(tmp, "layout")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    want = [fc.ctypes.sizeof(fc.BuildOpts)] + [getattr(fc.BuildOpts, f).offset for f, _ in fc.BuildOpts._fields_]
    assert [int(x) for x in out] == want


HANDLE_CALLS = [
    "fclsh_hash_sparse", "fclsh_query_batch_sparse", "fclsh_query_cost_sparse", "fclsh_query_batch",
    "fclsh_index_info", "fclsh_index_memory", "fclsh_index_params", "fclsh_hash", "fclsh_index_tables",
    "fclsh_index_table_keys", "fclsh_index_rebuild", "fclsh_index_rebuild_async", "fclsh_index_rebuild_timed",
    "fclsh_index_build_mode", "fclsh_query_collisions", "fclsh_query_cost", "fclsh_query_plain",
    "fclsh_query_batch_finish", "fclsh_query_batch_radii", "fclsh_query_reserve", "fclsh_query_batch_async",
    "fclsh_query_batch_noalloc", "fclsh_query_graph_create", "fclsh_index_set_tuning", "fclsh_index_get_tuning",
    "fclsh_index_set_schedule", "fclsh_index_get_schedule", "fclsh_autotune",
]


@pytest.mark.parametrize("name", HANDLE_CALLS)
def test_null_index_is_rejected(name):
    """Every call on an index checks its handle before any device work: a
    null handle gives FCLSH_EINVAL (here, with no GPU, nothing else runs)."""
    import ctypes

    fn = getattr(fc.lib(), name)
    assert fn.argtypes, f"{name}: no signature in the binding"
    scalars = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_float, ctypes.c_double)
    args = [0 if t in scalars else None for t in fn.argtypes]  # pointers null
    assert fn(*args) == fc.FCLSH_EINVAL, name


def test_bench_runs_on_one_gpu_only():
    # a multi-GPU request exits with a message before anything is set up
    import json
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert p.returncode == 2
    out = json.loads(p.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "exactly one GPU" in out["error"]


@pytest.mark.parametrize("flag", ["--batched", "--served"])
def test_bench_refuses_the_switched_off_sections(flag):
    # the two sections stay off the GPU: the benchmark exits with an error
    # before it imports torch or touches a device
    import json
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, os.path.join(root, "bench.py"), flag], capture_output=True, text=True,
                       timeout=60)
    assert p.returncode == 2
    assert "switched off" in json.loads(p.stdout.strip().splitlines()[-1])["error"]
