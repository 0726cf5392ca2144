"""The C-ABI library loads, exports every symbol include/crhyb.h declares, and its
host-only topology step (a0) agrees with the oracle.  CPU only: no call here
touches a device."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
import synth.workloads as wl
from oracle import cr

crh = pytest.importorskip("paper_2101_03777_amd")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "crhyb.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(cr_[A-Za-z_0-9]+)\s*\(", txt)))


def test_library_exports_header_symbols():
    lib = crh.load()
    names = header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(crh.EXPORTS) == names
    assert lib.cr_version().decode().startswith("crhyb")


def test_topology_matches_oracle_2d():
    coords, elems = synth.square_mesh(9, jitter=0.2, seed=1)
    t = crh.topology(coords, elems)
    m = cr.build_mesh(coords, elems)
    assert t["n_int_faces"] == m.nf
    assert sorted(t["perm"].tolist()) == list(range(m.nf))
    assert t["bandwidth_internal"] <= 4 * 9   # O(N) band on an N x N grid


def test_topology_matches_oracle_3d():
    coords, elems = synth.cube_mesh(3)
    t = crh.topology(coords, elems)
    m = cr.build_mesh(coords, elems)
    assert t["n_int_faces"] == m.nf
    assert sorted(t["perm"].tolist()) == list(range(m.nf))


def test_rcm_reduces_bandwidth_on_shuffled_mesh():
    """Reverse Cuthill-McKee on a randomly relabelled mesh recovers a narrow band
    (steady case: a transient mesh with aggregates takes the locality order of
    the coarse correction instead)."""
    coords, elems = synth.square_mesh(24)
    rng = np.random.default_rng(0)
    relabel = rng.permutation(len(coords))
    inv = np.argsort(relabel)
    c2 = coords[inv]
    e2 = relabel[elems].astype(np.int32)
    e2 = e2[rng.permutation(len(e2))]
    t = crh.topology(c2, e2, mu=0.0)
    nat = crh.topology(c2, e2, mu=0.0, renumber="natural")
    assert nat["bandwidth_internal"] == nat["bandwidth_canonical"]
    assert t["bandwidth_internal"] < 0.1 * t["bandwidth_canonical"]
    assert t["bandwidth_internal"] <= 4 * 24


def test_m1_partition_matches_oracle():
    ns = wl.ns_square(6)
    t = crh.topology(ns["coords"], ns["elems"], mu=0.0, nu=0.01, problem="ns")
    m = cr.build_mesh(ns["coords"], ns["elems"])
    in1, _ = cr.mis_partition(m)
    assert (t["m1"] == in1).all()
    assert not crh.topology(ns["coords"], ns["elems"], mu=1.0)["m1"].any()


def test_topology_errors():
    coords, elems = synth.square_mesh(2)
    with pytest.raises(crh.CRError) as e:
        crh.topology(coords, np.concatenate([elems, elems[:1]]))
    assert e.value.status == -3
    flat = coords.copy()
    flat[:, 1] = 0.0
    with pytest.raises(crh.CRError) as e:
        crh.topology(flat, elems)
    assert e.value.status == -3
    with pytest.raises(crh.CRError) as e:
        crh.topology(coords, elems, nu=0.0)
    assert e.value.status == -1
    with pytest.raises(crh.CRError) as e:
        crh.topology(coords, elems, k0=len(elems))
    assert e.value.status == -1
    bad = elems.copy()
    bad[0, 0] = len(coords) + 5
    with pytest.raises(crh.CRError) as e:
        crh.topology(coords, bad)
    assert e.value.status == -3
    # the Newton step is accepted in 3D as in 2D
    c3, e3 = synth.cube_mesh(1)
    t3 = crh.topology(c3, e3, mu=0.0, nu=0.01, problem="ns")
    assert t3["n_int_faces"] == 6 and t3["m1"].any()
    # a single triangle has no interior face
    with pytest.raises(crh.CRError) as e:
        crh.topology(coords[:3], np.array([[0, 1, 3]], dtype=np.int32) % 3)
    assert e.value.status == -3


def test_prepare_is_host_only():
    """cr_prepare (the host part of cr_assemble) runs without a device, with and
    without the aggregates of the coarse correction, and reports bad input."""
    lib = crh.load()
    coords, elems = synth.square_mesh(64, jitter=0.2, seed=3)  # 8192 elements: 64 aggregates
    for mu, problem in ((100.0, "stokes"), (0.0, "stokes"), (0.0, "ns")):
        p = crh.Prepared(coords, elems, mu=mu, nu=1.0, problem=problem)
        assert p.n_elements == len(elems) and p.dim == 2
        h = p.take()
        with pytest.raises(ValueError):
            p.take()
        lib.cr_prepared_destroy(h)
    c3, e3 = synth.cube_mesh(3)
    crh.Prepared(c3, e3, mu=10.0, nu=1.0)  # released by its destructor
    lib.cr_prepared_destroy(None)
    with pytest.raises(crh.CRError) as e:
        crh.Prepared(coords, elems, mu=1.0, nu=0.0)
    assert e.value.status == -1
    with pytest.raises(crh.CRError) as e:
        crh.Prepared(coords[:3], np.array([[0, 1, 2]], dtype=np.int32), mu=1.0, nu=1.0)
    assert e.value.status == -3


def test_one_hip_runtime_in_the_process():
    """Loading the library before torch is imported still leaves one HIP runtime
    in the process (the one torch brings), whichever import comes first."""
    import subprocess
    import sys
    code = ("import paper_2101_03777_amd as crh\n"
            "crh.load()\n"
            "import torch\n"
            "libs = set()\n"
            "for line in open('/proc/self/maps'):\n"
            "    f = line.split()\n"
            "    if len(f) >= 6 and 'libamdhip64' in f[-1]:\n"
            "        libs.add(f[-1])\n"
            "print(len(libs))\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip().splitlines()[-1] == "1"
