"""CPU checks of the C interface: the library loads, exports every function
that include/sel.h declares, and its host-side mesh ingest validates input
(no device call is made here)."""
import ctypes
import os
import re

import numpy as np
import pytest

from conftest import ROOT
from paper_2509_19171_amd import inputs as I
from paper_2509_19171_amd import sel

HEADER = os.path.join(ROOT, "include", "sel.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sel_[a-z_0-9]+)\s*\(", txt)))


def test_exports_every_declared_symbol():
    lib = sel.load()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    # and nothing of the oracle is linked in
    assert not hasattr(lib, "oracle_step")
    assert "gfx950" in sel.version()


def test_mesh_ingest_groups():
    m = I.box_mesh(2, 3, (4, 3), (0, 0), (1, 1), (True, False), wall_tags={1: (1, 2)},
                   wall_u=[[0, 0], [0.1, 0]])
    sm = sel.Mesh.from_inputs(m)
    info = sm.info()
    assert info["np"] == 16 and info["E"] == 12
    assert info["boundary_nodes_per_element"] == 16 - 4
    # unique nodes of a 4x3 element periodic-in-x channel at N = 3: (4*3) x (3*3 + 1)
    assert info["unique_nodes"] == len(np.unique(m.gid)) == 12 * 10
    assert info["wall_faces"] == 8


def test_mesh_ingest_rejects_bad_input():
    m = I.box_mesh(2, 3, (2, 2), (0, 0), (1, 1), (True, True))
    gid = m.gid.copy()
    gid[0, 5] = gid[1, 5]  # share an interior node
    with pytest.raises(sel.SelError) as ex:
        sel.Mesh(2, 3, m.xyz, gid, m.face_tag)
    assert ex.value.code == sel.SEL_EINVAL
    gid = m.gid.copy()
    gid[0, 0] = m.E * m.np_  # out of range
    with pytest.raises(sel.SelError):
        sel.Mesh(2, 3, m.xyz, gid, m.face_tag)
    ft = m.face_tag.copy()
    ft[0, 0] = 3  # tag beyond ntags
    with pytest.raises(sel.SelError):
        sel.Mesh(2, 3, m.xyz, m.gid, ft)
    with pytest.raises(sel.SelError) as ex:
        sel.Mesh(4, 3, m.xyz, m.gid, m.face_tag)
    assert ex.value.code == sel.SEL_EINVAL
    with pytest.raises(sel.SelError) as ex:
        sel.Mesh(2, 1, m.xyz, m.gid, m.face_tag)
    assert ex.value.code == sel.SEL_EUNSUPPORTED


def test_workspace_bytes_and_param_checks():
    c = I.case_tgv3d(nel=2, N=7, steps=0)
    sm = sel.Mesh.from_inputs(c.mesh)
    p64 = sel.params_from_case(c, "fp64")
    p32 = sel.params_from_case(c, "fp32dev")
    b64 = sm.workspace_bytes(p64)
    b32 = sm.workspace_bytes(p32)
    info = sm.info()
    G = info["unique_nodes"]
    assert b64 > 4 * 27 * G * 8 and b32 > 4 * 27 * G * 4 and b32 < b64
    bad = sel.params_from_case(c, "fp64")
    bad.Q = 9
    with pytest.raises(sel.SelError):
        sm.workspace_bytes(bad)
    bad = sel.params_from_case(c, "fp64")
    bad.nu = -1.0
    with pytest.raises(sel.SelError):
        sm.workspace_bytes(bad)
    bad = sel.params_from_case(c, "fp64")
    bad.filter_kc = 7
    with pytest.raises(sel.SelError):
        sm.workspace_bytes(bad)
    msg = sel.load().sel_last_error().decode()
    assert "filter_kc" in msg


def test_binding_refuses_missing_library(monkeypatch, tmp_path):
    monkeypatch.setattr(sel, "_lib", None)
    monkeypatch.setattr(sel, "LIB_PATH", str(tmp_path / "libsel.so"))
    with pytest.raises(RuntimeError):
        sel.load()


def test_mesh_create_dg_ingest():
    """The discontinuous coupling shares no node, and faces must pair up."""
    m = I.box_mesh(2, 4, (3, 2), (0, 0), (1, 1), (True, True))
    cg = sel.Mesh.from_inputs(m).info()
    dg = sel.Mesh.from_inputs(m, "dg").info()
    assert cg["unique_nodes"] < m.E * m.np_
    assert dg["unique_nodes"] == m.E * m.np_
    assert dg["groups"] == m.E * dg["boundary_nodes_per_element"]
    # walls are not interfaces: a channel with two wall sides is accepted
    ch = I.box_mesh(3, 3, (2, 2, 2), (0, 0, 0), (1, 1, 1), (True, False, True), wall_tags={1: (1, 1)},
                    wall_u=[[0, 0, 0]])
    assert sel.Mesh.from_inputs(ch, "dg").info()["wall_faces"] == 8
    # one element along a periodic direction: a face repeats a node id
    one = I.box_mesh(2, 4, (1, 3), (0, 0), (1, 1), (True, True))
    with pytest.raises(sel.SelError) as ex:
        sel.Mesh.from_inputs(one, "dg")
    assert ex.value.code == sel.SEL_EINVAL
    sel.Mesh.from_inputs(one)  # the continuous coupling accepts it
    # open boundary faces have no partner
    opn = I.box_mesh(2, 4, (2, 2), (0, 0), (1, 1), (False, False), wall_tags={0: (0, 0), 1: (0, 0)})
    with pytest.raises(sel.SelError) as ex:
        sel.Mesh.from_inputs(opn, "dg")
    assert ex.value.code == sel.SEL_EINVAL


def test_mesh_ingest_rejects_inconsistent_copies():
    """Copies sharing a node id must coincide, or differ by the mesh's periodic
    translations (Sec. 2.2: the continuous coupling identifies them)."""
    m = I.box_mesh(3, 3, (2, 2, 2), (0, 0, 0), (1, 1, 1), (True, True, False), wall_tags={2: (1, 2)},
                   wall_u=[[0, 0, 0], [0.1, 0, 0]])
    sel.Mesh.from_inputs(m)
    # a node inside the face between elements 0 and 1 moved in one copy only
    n1 = 4
    p = 3 + n1 * 1 + n1 * n1 * 2  # (i, j, k) = (3, 1, 2): r+ face of element 0, off its edges
    xyz = m.xyz.copy()
    xyz[0, p, 1] += 0.01
    with pytest.raises(sel.SelError) as ex:
        sel.Mesh(3, 3, xyz, m.gid, m.face_tag, m.wall_u)
    assert ex.value.code == sel.SEL_EINVAL and "displaced" in str(ex.value)
    # two ids swapped inside that face: the copies no longer coincide
    gid = m.gid.copy()
    q = 3 + n1 * 2 + n1 * n1 * 1
    gid[0, p], gid[0, q] = m.gid[0, q], m.gid[0, p]
    with pytest.raises(sel.SelError) as ex:
        sel.Mesh(3, 3, m.xyz, gid, m.face_tag, m.wall_u)
    assert ex.value.code == sel.SEL_EINVAL
    # a corner copy moved (edges and corners are checked against the face translations)
    xyz = m.xyz.copy()
    xyz[3, 0, 0] += 0.01
    with pytest.raises(sel.SelError) as ex:
        sel.Mesh(3, 3, xyz, m.gid, m.face_tag, m.wall_u)
    assert ex.value.code == sel.SEL_EINVAL and "coincide" in str(ex.value)


def test_mesh_ingest_accepts_periodic_translations():
    """Periodic copies differ by translations (here of a skewed box, so the
    translations are not axis-aligned); edges and corners combine them. A
    single element along a periodic direction shares nodes with itself."""
    A = np.array([[1.0, 0.3, 0.1], [-0.2, 0.9, 0.2], [0.1, 0.05, 1.1]])
    m = I.box_mesh(3, 3, (2, 1, 3), (0, 0, 0), (1, 1, 1), (True, True, True), warp=lambda x: x @ A.T)
    sel.Mesh.from_inputs(m)
    sel.Mesh.from_inputs(I.box_mesh(2, 5, (1, 1), (0, 0), (1, 1), (True, True)))
    sel.Mesh.from_inputs(I.case_pipe(N=3, nsq=2, nrad=2, nax=2, L=2.0).mesh)


def test_mesh_ingest_rejects_shared_wall_face():
    """A wall face (Sec. 2.2.1) lies on the domain boundary: none of its nodes
    off its edges may be shared with another face."""
    m = I.box_mesh(2, 4, (2, 2), (0, 0), (1, 1), (True, False), wall_tags={1: (1, 2)},
                   wall_u=[[0, 0], [0.1, 0]])
    sel.Mesh.from_inputs(m)
    ft = m.face_tag.copy()
    ft[0, 3] = 1  # the s+ face of element 0 is the interface with element 2
    with pytest.raises(sel.SelError) as ex:
        sel.Mesh(2, 4, m.xyz, m.gid, ft, m.wall_u)
    assert ex.value.code == sel.SEL_EINVAL and "wall face" in str(ex.value)


def test_compiled_orders_and_refusals():
    """3D orders N 2..8 run one thread per element node; D3Q19 also at
    N = 12 (2197 nodes, the paper's highest Taylor-Green order), with several
    nodes per thread. Other orders and lattices, and the closure at N = 12,
    are refused with SEL_EUNSUPPORTED before any device call."""
    c12 = I.case_tgv3d(nel=1, N=12, Q=19, steps=0)
    m12 = sel.Mesh.from_inputs(c12.mesh)
    for prec in ("fp64", "fp32dev"):
        assert m12.workspace_bytes(sel.params_from_case(c12, prec)) > 0
    c8 = I.case_tgv3d(nel=1, N=8, Q=19, steps=0)
    assert sel.Mesh.from_inputs(c8.mesh).workspace_bytes(sel.params_from_case(c8, "fp32dev")) > 0
    refused = [(I.case_tgv3d(nel=1, N=12, Q=27, steps=0), None), (I.case_tgv3d(nel=1, N=10, Q=19, steps=0), None),
               (c12, np.zeros(sel.closure_len(), dtype=np.float32))]
    for c, blob in refused:
        p = sel.params_from_case(c, "fp32dev")
        if blob is not None:
            p._closure_blob = blob
            p.closure = blob.ctypes.data
            p.closure_len = blob.size
        with pytest.raises(sel.SelError) as ex:
            sel.Mesh.from_inputs(c.mesh).workspace_bytes(p)
        assert ex.value.code == sel.SEL_EUNSUPPORTED, (c.N, c.Q)
    c12b = I.case_tgv3d(nel=2, N=12, Q=19, steps=0)  # two elements per periodic direction
    with pytest.raises(sel.SelError) as ex:
        sel.Mesh.from_inputs(c12b.mesh, "dg").workspace_bytes(sel.params_from_case(c12b, "fp64"))
    assert ex.value.code == sel.SEL_EUNSUPPORTED
