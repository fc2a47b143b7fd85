"""AddressSanitizer and UndefinedBehaviorSanitizer builds of host code, run on
the CPU: the FP64 oracle (``oracle/sel_oracle.c``) over a few small cases
(2D and 3D, walls, periodic boxes, both couplings, both time-marching forms,
a per-node force), and the library's mesh ingest and table construction
(``csrc/mesh.cpp``, ``csrc/tables.cpp``; host code only, compiled with g++)
on valid meshes and on meshes each validation rule rejects. Any sanitizer
report makes the driver exit non-zero."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

from conftest import ROOT
from paper_2509_19171_amd import inputs as I

SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
HERE = os.path.dirname(os.path.abspath(__file__))
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="1")


@pytest.fixture(scope="module")
def build_dir(tmp_path_factory):
    if shutil.which("gcc") is None or shutil.which("g++") is None:
        pytest.skip("gcc/g++ not available")
    d = tmp_path_factory.mktemp("sanitize")
    subprocess.run(["gcc", "-std=c11", "-D_DEFAULT_SOURCE"] + SAN +
                   ["-o", str(d / "oracle_main"), os.path.join(HERE, "sanitize", "oracle_main.c"),
                    os.path.join(ROOT, "oracle", "sel_oracle.c"), "-lm"], check=True)
    csrc = os.path.join(ROOT, "paper_2509_19171_amd", "csrc")
    subprocess.run(["g++", "-x", "c++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    "-I" + os.path.join(ROOT, "include"), "-I" + csrc] + SAN +
                   ["-o", str(d / "ingest_main"), os.path.join(HERE, "sanitize", "ingest_main.cpp"),
                    os.path.join(csrc, "mesh.cpp"), os.path.join(csrc, "tables.cpp")], check=True)
    return d


def _write_mesh(path, m):
    with open(path, "wb") as fh:
        np.array([m.dim, m.N, m.E, m.wall_u.shape[0]], dtype=np.int64).tofile(fh)
        np.ascontiguousarray(m.xyz, dtype=np.float64).tofile(fh)
        np.ascontiguousarray(m.gid, dtype=np.int64).tofile(fh)
        np.ascontiguousarray(m.face_tag, dtype=np.int32).tofile(fh)
        np.ascontiguousarray(m.wall_u, dtype=np.float64).tofile(fh)


def _write_case(path, c):
    ftype = {None: 0, "none": 0, "quad": 1, "exp": 2}[c.filter]
    ntags = c.wall_u.shape[0]
    wu = c.wall_u if ntags else np.zeros((1, c.dim))
    with open(path, "wb") as fh:
        np.array([c.dim, c.N, c.E, c.Q, ntags, ftype, c.filter_kc, {"ssprk3": 0, "printed4": 1}[c.rk],
                  {"cg": 0, "dg": 1}[c.coupling]], dtype=np.int64).tofile(fh)
        g = list(c.g) + [0.0] * (3 - len(c.g))
        np.array([c.rho0, c.nu, c.dt] + g[:3] + [c.filter_amp, c.filter_order], dtype=np.float64).tofile(fh)
        np.ascontiguousarray(c.xyz, dtype=np.float64).tofile(fh)
        np.ascontiguousarray(c.gid, dtype=np.int64).tofile(fh)
        np.ascontiguousarray(c.face_tag, dtype=np.int32).tofile(fh)
        np.ascontiguousarray(wu, dtype=np.float64).tofile(fh)
        np.ascontiguousarray(c.rho, dtype=np.float64).tofile(fh)
        np.ascontiguousarray(c.u, dtype=np.float64).tofile(fh)


def _run(cmd):
    r = subprocess.run(cmd, env=ENV, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, \
        r.stderr[-4000:]
    return r.stdout


def _oracle_cases():
    c1 = I.case_couette(nelx=2, nely=2, N=4, curved=True, filt="quad")
    c2 = I.case_tgv3d(nel=2, N=3, Q=27, Re=200.0, steps=0, filt="exp")
    m3 = I.box_mesh(3, 3, (2, 2, 2), (0, 0, 0), (1, 1, 1), (True, False, True), wall_tags={1: (1, 2)},
                    wall_u=[[0, 0, 0], [0.02, 0, 0.01]])
    r3, u3 = I.rest_fields(m3.xyz)
    c3 = I.Case("box3d_q19", m3, 19, 1.0, 0.01, I.stable_dt(m3), r3, u3, 0, g=(1e-3, 0.0, 0.0), filter="quad",
                filter_kc=2, filter_amp=0.1, rk="printed4")
    c4 = I.case_tgv2d(nel=3, N=4, steps=0)
    c4.coupling = "dg"
    m5 = I.box_mesh(2, 5, (1, 1), (0, 0), (2 * math.pi, 2 * math.pi), (True, True))
    r5, u5 = I.tgv2d_fields(m5.xyz, 0.05)
    c5 = I.Case("single", m5, 9, 1.0, 0.01, I.stable_dt(m5), r5, u5, 0)
    return {"couette_curved": c1, "tgv3d_q27": c2, "box3d_q19_printed4": c3, "tgv2d_dg": c4, "single_element": c5}


@pytest.mark.parametrize("name", list(_oracle_cases()))
def test_oracle_under_sanitizers(build_dir, tmp_path, name):
    c = _oracle_cases()[name]
    f = tmp_path / "case.bin"
    _write_case(f, c)
    out = _run([str(build_dir / "oracle_main"), str(f), "3"])
    assert out.startswith("ok")


def _ingest_cases():
    ok = {
        "channel2d": I.box_mesh(2, 3, (4, 3), (0, 0), (1, 1), (True, False), wall_tags={1: (1, 2)},
                                wall_u=[[0, 0], [0.1, 0]]),
        "single2d": I.box_mesh(2, 4, (1, 1), (0, 0), (1, 1), (True, True)),
        "skew3d": I.box_mesh(3, 3, (2, 1, 2), (0, 0, 0), (1, 1, 1), (True, True, True),
                             warp=lambda x: x @ np.array([[1.0, 0.3, 0.1], [-0.2, 0.9, 0.2], [0.1, 0.05, 1.1]]).T),
        "pipe": I.case_pipe(N=3, nsq=2, nrad=2, nax=2, L=2.0).mesh,
    }
    out = {k: (m, 0, 0) for k, m in ok.items()}
    out["channel2d_dg"] = (ok["channel2d"], 0, 1)
    bad = I.box_mesh(3, 3, (2, 2, 2), (0, 0, 0), (1, 1, 1), (True, True, False), wall_tags={2: (1, 2)},
                     wall_u=[[0, 0, 0], [0.1, 0, 0]])
    moved = I.Mesh(3, 3, bad.xyz.copy(), bad.gid, bad.face_tag, bad.wall_u)
    moved.xyz[0, 3 + 4 + 32, 1] += 0.01
    out["moved_face_node"] = (moved, -1, 0)
    corner = I.Mesh(3, 3, bad.xyz.copy(), bad.gid, bad.face_tag, bad.wall_u)
    corner.xyz[3, 0, 0] += 0.01
    out["moved_corner"] = (corner, -1, 0)
    ft = ok["channel2d"].face_tag.copy()
    ft[0, 3] = 1
    out["shared_wall_face"] = (I.Mesh(2, 3, ok["channel2d"].xyz, ok["channel2d"].gid, ft, ok["channel2d"].wall_u),
                               -1, 0)
    gid = ok["channel2d"].gid.copy()
    gid[0, 0] = ok["channel2d"].E * 16
    out["gid_range"] = (I.Mesh(2, 3, ok["channel2d"].xyz, gid, ok["channel2d"].face_tag, ok["channel2d"].wall_u),
                        -1, 0)
    one = I.box_mesh(2, 4, (1, 3), (0, 0), (1, 1), (True, True))
    out["dg_repeated_id"] = (one, -1, 1)
    return out


@pytest.mark.parametrize("name", list(_ingest_cases()))
def test_ingest_under_sanitizers(build_dir, tmp_path, name):
    m, expect, dg = _ingest_cases()[name]
    f = tmp_path / "mesh.bin"
    _write_mesh(f, m)
    out = _run([str(build_dir / "ingest_main"), str(f), str(expect), str(dg)])
    assert out.startswith("ok")
