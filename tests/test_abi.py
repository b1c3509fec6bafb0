"""Host-side checks of the C-ABI library (no GPU): it loads, exports every symbol
declared in include/etpic.h, and its host canonicalisation of a mesh agrees
bit for bit with the oracle's and the input generator's numbering."""
import os
import re

import numpy as np
import pytest

from paper_2208_12795_amd import etpic, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "etpic.h")).read()
    return sorted(set(re.findall(r"\b(etpic_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = etpic.lib()
    declared = header_symbols()
    assert len(declared) >= 12
    for name in declared:
        assert hasattr(L, name), name
    assert sorted(etpic.EXPORTS) == declared


@pytest.mark.parametrize("n", [(1, 1, 1), (3, 2, 4), (5, 5, 5)])
def test_canonical_numbering_matches_oracle(ora, n):
    xyz, tv = synth.kuhn_mesh(n, (1.0, 2.0, 1.5), 0.1, np.random.default_rng(5))
    cnt, edges, faces = etpic.mesh_canonical(xyz, tv)
    M = ora.OracleMesh(xyz, tv)
    assert tuple(cnt) == (M.nv, M.ne, M.nf, M.nt)
    assert np.array_equal(edges, M.edges())
    assert np.array_equal(faces, M.faces())
    assert np.array_equal(edges, synth.mesh_edges(tv, xyz.shape[0]))


def test_canonical_rejects_bad_meshes():
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1.0], [1, 1, 1.0]])
    with pytest.raises(etpic.EtpicError) as e:
        etpic.mesh_canonical(xyz, np.array([[0, 2, 1, 3]], np.int32))
    assert e.value.code == etpic.EMESH
    with pytest.raises(etpic.EtpicError) as e:
        etpic.mesh_canonical(xyz, np.array([[0, 1, 2, 9]], np.int32))
    assert e.value.code == etpic.EINVAL
    flat = xyz.copy()
    flat[3] = [1, 1, 0]
    with pytest.raises(etpic.EtpicError) as e:
        etpic.mesh_canonical(flat, np.array([[0, 1, 2, 3]], np.int32))
    assert e.value.code == etpic.EMESH
    # three tets sharing one face -> non-manifold
    xyz3 = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1.0], [0.2, 0.2, -1], [0.3, 0.3, 2.0]])
    tv3 = np.array([[0, 1, 2, 3], [0, 1, 2, 4], [0, 1, 2, 5]], np.int32)
    with pytest.raises(etpic.EtpicError) as e:
        etpic.mesh_canonical(xyz3, tv3)
    assert e.value.code == etpic.EMESH


def test_no_cpu_fallback_without_library(monkeypatch, tmp_path):
    """The binding refuses to run when the HIP library is absent."""
    monkeypatch.setattr(etpic, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(etpic, "_lib", None)
    with pytest.raises(RuntimeError):
        etpic.lib()


def test_binding_constants_match_header():
    """Every ETPIC_* enum value of the header has the same value in the binding."""
    txt = open(os.path.join(ROOT, "include", "etpic.h")).read()
    vals = dict((k, int(v.rstrip("u"))) for k, v in re.findall(r"\bETPIC_([A-Z0-9_]+)\s*=\s*(-?\d+u?)", txt))
    assert len(vals) >= 15
    alias = {"DEV_HOPCAP": "DEV_HOPCAP", "HOP_CAP": "HOP_CAP"}
    for k, v in vals.items():
        name = alias.get(k, k.replace("STEP_", "STEP_"))
        assert getattr(etpic, name) == v, k
    assert etpic.HOP_CAP == int(re.search(r"ETPIC_HOP_CAP\s+(\d+)", txt).group(1))


def test_workspace_and_mesh_sizes_are_host_queries():
    """The size queries of the caller-owned buffers run on the host: the
    context workspace is a fixed size (two walk queues of 2^23 entries and a
    few words), the mesh buffer grows with the mesh and reports the canonical
    counts; a bad mesh is refused before any size is given."""
    import ctypes as C
    L = etpic.lib()
    b = C.c_size_t(0)
    assert L.etpic_workspace_bytes(C.byref(b)) == 0
    assert b.value >= 2 * 4 * (1 << 23)
    sizes = []
    for n in [(2, 2, 2), (4, 3, 5)]:
        xyz, tv = synth.kuhn_mesh(n, (1.0, 1.0, 1.0), 0.1, np.random.default_rng(1))
        cnt = np.zeros(4, dtype=np.int64)
        mb = C.c_size_t(0)
        rc = L.etpic_mesh_sizes(xyz.shape[0], xyz.ctypes.data_as(C.POINTER(C.c_double)), tv.shape[0],
                                np.ascontiguousarray(tv, np.int32).ctypes.data_as(C.POINTER(C.c_int32)),
                                cnt.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(mb))
        assert rc == 0
        ref, _, _ = etpic.mesh_canonical(xyz, tv)
        assert tuple(cnt) == tuple(ref)
        nt = tv.shape[0]
        # at least the per-tet rows it holds: topology 80 B, gradients 96 B, coefficient table 192 B,
        # two slot buffers 2 x 64 B per tet
        assert mb.value >= nt * (80 + 96 + 192 + 128)
        sizes.append(mb.value)
    assert sizes[1] > sizes[0]
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1.0]])
    cnt = np.zeros(4, dtype=np.int64)
    bad = np.array([[0, 2, 1, 3]], np.int32)
    rc = L.etpic_mesh_sizes(4, xyz.ctypes.data_as(C.POINTER(C.c_double)), 1,
                            bad.ctypes.data_as(C.POINTER(C.c_int32)), cnt.ctypes.data_as(C.POINTER(C.c_int64)),
                            C.byref(b))
    assert rc == etpic.EMESH


def test_vector_checker_refuses_before_any_call():
    """The binding's device-vector check (length, dtype, contiguity, device)
    raises EINVAL itself; NULL passes only where the argument is optional."""
    import torch
    from paper_2208_12795_amd import etpic as E
    assert E._vec(None, 10, "rho") is None
    for bad in (lambda: E._vec(None, 10, "dG", optional=False),
                lambda: E._vec(torch.zeros(10, dtype=torch.float64), 10, "dG"),     # host memory
                lambda: E._vec(np.zeros(10), 10, "dG")):
        with pytest.raises(E.EtpicError) as ei:
            bad()
        assert ei.value.code == E.EINVAL and "dG" in str(ei.value)
