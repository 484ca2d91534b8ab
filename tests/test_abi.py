"""The C-ABI library loads and exports what include/ssj.h declares (no GPU)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ssj.h")
LIB = os.path.join(ROOT, "paper_1812_09141_amd", "libssj.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ssj_[a-z_]+)\s*\(", text)))


def exported_symbols():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    return {line.split()[-1] for line in out.splitlines() if line.strip()}


@pytest.fixture(scope="module")
def built():
    if not os.path.exists(LIB):
        from paper_1812_09141_amd import build
        build.build()
    return LIB


def test_header_declares_core_calls():
    names = declared_functions()
    for n in ["ssj_init", "ssj_upload_collection", "ssj_verify", "ssj_verify_device",
              "ssj_stream_submit", "ssj_stream_poll"]:
        assert n in names


def test_every_declared_symbol_exported(built):
    exp = exported_symbols()
    missing = [n for n in declared_functions() if n not in exp]
    assert not missing, missing


def test_binding_names_match_header(built):
    import paper_1812_09141_amd.ssj as ssj
    assert sorted(ssj.EXPORTED) == declared_functions()
    lib = ssj.load_library()
    for n in ssj.EXPORTED:
        assert hasattr(lib, n)
        assert hasattr(ssj, n)


def test_library_independent_of_oracle(built):
    exp = exported_symbols()
    assert not any(s.startswith("ssjref_") for s in exp)
    needed = subprocess.run(["readelf", "-d", LIB], capture_output=True, text=True).stdout
    assert "ssj_oracle" not in needed and "allpairs" not in needed


def test_init_without_gpu_fails_cleanly(built):
    import torch
    import paper_1812_09141_amd.ssj as ssj
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(ssj.SsjError) as e:
        ssj.ssj_init(0)
    assert e.value.code == ssj.SSJ_EDEVICE


def test_constants_match_header():
    import paper_1812_09141_amd.ssj as ssj
    text = open(HEADER).read()
    for name in ["SSJ_OK", "SSJ_PENDING", "SSJ_EINVAL", "SSJ_ENOMEM", "SSJ_ETRUNC", "SSJ_EAGAIN",
                 "SSJ_EDEVICE", "SSJ_ENOTFOUND"]:
        m = re.search(name + r"\s*=\s*(-?\d+)", text)
        assert m and int(m.group(1)) == getattr(ssj, name)
    m = re.search(r"SSJ_CLASS_BOUNDS\s*\{([^}]*)\}", text)
    vals = tuple(int(v.strip(), 0) for v in m.group(1).split(","))
    assert vals == ssj.SSJ_CLASS_BOUNDS
    assert int(re.search(r"SSJ_N_CLASSES\s+(\d+)", text).group(1)) == ssj.SSJ_N_CLASSES
    for name in ["SSJ_SIM_JACCARD", "SSJ_SIM_COSINE", "SSJ_SIM_DICE", "SSJ_SIM_OVERLAP"]:
        m = re.search(r"#define\s+" + name + r"\s+(\d+)", text)
        assert m and int(m.group(1)) == getattr(ssj, name)


def test_request_struct_matches_header():
    # the batch request struct ends with the similarity function
    import ctypes
    import paper_1812_09141_amd.ssj as ssj
    text = open(HEADER).read()
    body = re.search(r"typedef struct \{([^}]*)\} ssj_request;", text).group(1)
    fields = [ln.strip().rstrip(";").split()[-1].lstrip("*") for ln in body.strip().splitlines()
              if ln.strip() and not ln.strip().startswith("/")]
    assert fields == [f[0] for f in ssj.ssj_request._fields_]
    assert ctypes.sizeof(ssj.ssj_request) == 64


def test_plan_struct_matches_header():
    # field names and order of the plan struct in the header and the binding
    import ctypes
    import paper_1812_09141_amd.ssj as ssj
    text = open(HEADER).read()
    body = re.search(r"typedef struct \{([^}]*)\} ssj_plan;", text).group(1)
    fields = [m.group(1) for m in re.finditer(r"\bint\s+(\w+)\s*(?:\[[^\]]*\])?\s*;",
                                                re.sub(r"/\*.*?\*/", "", body, flags=re.S))]
    assert fields == [f[0] for f in ssj.ssj_plan._fields_]
    assert ctypes.sizeof(ssj.ssj_plan) == 4 * (8 + ssj.SSJ_N_CLASSES)


def test_groups_of_runs():
    """The binding's grouped form of flat pairs: one group per run of equal r,
    ends exclusive, s ids in order (repeated probes make separate groups)."""
    import numpy as np
    import paper_1812_09141_amd.ssj as ssj
    pairs = np.array([[3, 1], [3, 2], [1, 5], [1, 5], [3, 0], [7, 7]], np.int32)
    g, s = ssj.groups_of(pairs)
    assert g.tolist() == [[3, 2], [1, 4], [3, 5], [7, 6]]
    assert s.tolist() == [1, 2, 5, 5, 0, 7]
    g0, s0 = ssj.groups_of(np.zeros((0, 2), np.int32))
    assert g0.shape == (0, 2) and s0.shape == (0,)


def test_group_request_layout():
    """ssj_group_request in the binding matches the C layout of include/ssj.h
    (pointers and int64 fields in declaration order, then an int32; 80 bytes)."""
    import ctypes
    from paper_1812_09141_amd import ssj as S
    t = S.ssj_group_request
    names = [f[0] for f in t._fields_]
    assert names == ["d_groups", "n_groups", "d_cand", "n_cand", "t_num", "t_den", "d_out", "out_cap",
                     "d_count", "sim"]
    assert [getattr(t, n).offset for n in names] == [0, 8, 16, 24, 32, 40, 48, 56, 64, 72]
    assert ctypes.sizeof(t) == 80
    src = open(os.path.join(ROOT, "include", "ssj.h")).read()
    body = src[src.index("typedef struct {\n    const ssj_group* d_groups;"):]
    body = body[:body.index("} ssj_group_request;")]
    assert [ln.strip().rstrip(";").split()[-1].lstrip("*") for ln in body.splitlines()[1:] if ln.strip()] == names
