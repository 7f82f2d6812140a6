"""CPU tests of the library's host code (mesh, A_s, ordering, factor, sweep plan).

A test driver built from the library's host sources replays the GPU sweeps'
index arithmetic with bounds checks; its outputs are compared with the oracle.
"""
import os
import subprocess
import tempfile

import numpy as np
import pytest

import workloads as W
from oracle import model as om
from parity_helpers import robot_scene, ragged_scene

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2101_05917_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("host") / "host_check")
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-o", out,
           os.path.join(HERE, "host", "host_check.cpp"),
           os.path.join(CSRC, "host_mesh.cpp"), os.path.join(CSRC, "factor.cpp")]
    subprocess.run(cmd, check=True)
    return out


@pytest.fixture(scope="module")
def sanitized_driver(tmp_path_factory):
    """The same driver built with AddressSanitizer and UndefinedBehaviorSanitizer
    (host code only: g++, no device code): any out-of-bounds access, use after
    free, leak or undefined operation in the mesh, ordering, factor or sweep-plan
    code aborts the run."""
    out = str(tmp_path_factory.mktemp("host_asan") / "host_check_asan")
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fopenmp", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-o", out,
           os.path.join(HERE, "host", "host_check.cpp"),
           os.path.join(CSRC, "host_mesh.cpp"), os.path.join(CSRC, "factor.cpp")]
    subprocess.run(cmd, check=True)
    return out


def write_input(path, sc, leaf_max, sep_max, rhs=None):
    with open(path, "wb") as f:
        np.array([len(sc.cells)], np.int64).tofile(f)
        np.asarray(sc.cells, np.int32).tofile(f)
        np.asarray(sc.youngs, np.float64).tofile(f)
        np.array([len(sc.fixed_nodes)], np.int64).tofile(f)
        np.asarray(sc.fixed_nodes, np.int32).reshape(-1).tofile(f)
        ov = [sc.dx, sc.rho, sc.nu, sc.h, *sc.gravity, *sc.origin, sc.contact_k,
              sc.friction_mu, sc.friction_eps, sc.muscle_k, *sc.fiber]
        np.asarray(ov, np.float64).tofile(f)
        np.array([leaf_max, sep_max], np.int32).tofile(f)
        if rhs is not None:
            np.array([len(rhs)], np.int64).tofile(f)
            np.asarray(rhs, np.float64).tofile(f)


def run_driver(driver, sc, rhs, leaf_max=64, sep_max=2048):
    with tempfile.TemporaryDirectory() as d:
        fin, fout = os.path.join(d, "in.bin"), os.path.join(d, "out.bin")
        write_input(fin, sc, leaf_max, sep_max, rhs)
        res = subprocess.run([driver, fin, fout], capture_output=True, text=True)
        assert res.returncode == 0, res.stderr
        raw = open(fout, "rb").read()
    off = 0

    def take(dtype, n):
        nonlocal off
        a = np.frombuffer(raw, dtype=dtype, count=n, offset=off)
        off += a.nbytes
        return a

    N, nf, nnz, nsn, nlev, packed, nfwd, nbwd = take(np.int64, 8)
    out = {"N": N, "nf": nf, "n_supernodes": nsn, "n_levels": nlev, "packed_nnz": packed}
    out["ijk"] = take(np.int32, 3 * N).reshape(N, 3)
    out["mass"] = take(np.float64, N)
    out["free_nodes"] = take(np.int32, nf)
    ptr = take(np.int64, nf + 1)
    col = take(np.int32, nnz)
    val = take(np.float64, nnz)
    out["A"] = (ptr, col, val)
    out["x"] = take(np.float64, len(rhs) * 3 * N).reshape(len(rhs), 3, N)
    return out


CASES = {
    "c1": lambda: W.config("c1"),
    "c2": lambda: W.config("c2"),
    "robot": robot_scene,
    "ragged": ragged_scene,
    "free_block": lambda: W.dropped_block(6, 5, 4, steps=1),
    "one_voxel": lambda: W.dropped_block(1, 1, 1, steps=1),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("leaf,sep", [(64, 2048), (8, 16), (4096, 2048)])
def test_host_mesh_matrix_and_solve(driver, name, leaf, sep):
    sc = CASES[name]()
    o = om.Model(sc)
    rng = np.random.default_rng(0)
    rhs = rng.standard_normal((2, 3, o.N))
    out = run_driver(driver, sc, rhs, leaf, sep)
    assert np.array_equal(out["ijk"], o.mesh.node_ijk)
    assert np.allclose(out["mass"], o.m, rtol=1e-15, atol=0)
    # A_s equals each coordinate block of the oracle's A (free nodes)
    free_nodes = np.nonzero(o.free[0::3])[0]
    assert np.array_equal(out["free_nodes"], free_nodes)
    ptr, col, val = out["A"]
    nf = len(free_nodes)
    As = np.zeros((nf, nf))
    for i in range(nf):
        As[i, col[ptr[i]:ptr[i + 1]]] = val[ptr[i]:ptr[i + 1]]
    Af = o.A.toarray()
    for c in range(3):
        blk = Af[3 * free_nodes + c][:, 3 * free_nodes + c]
        assert np.abs(As - blk).max() <= 1e-12 * np.abs(blk).max()
    # no coupling between coordinates in the oracle's A (Kronecker structure)
    off = Af[0::3][:, 1::3]
    assert np.abs(off).max() == 0.0
    # the replayed sweeps solve A x = b on free nodes
    for k in range(len(rhs)):
        b = rhs[k].T.reshape(-1)
        ref = np.zeros(3 * o.N)
        ref[o.free] = o.solve_A(b[o.free])
        got = out["x"][k].T.reshape(-1)
        assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
        assert np.all(got[o.fixed] == 0.0)


@pytest.mark.slow
def test_host_solve_large_block_residual(driver):
    """A block large enough for the many-leaf kernels (>= 256 leaf supernodes):
    replayed sweeps solve A_s x = b to round-off (checked with the driver's A_s)."""
    sc = W.dropped_block(48, 24, 24, steps=1)
    N = len(W.present_nodes(sc.cells))
    rhs = np.random.default_rng(3).standard_normal((1, 3, N))
    out = run_driver(driver, sc, rhs)
    ptr, col, val = out["A"]
    nf = out["nf"]
    import scipy.sparse as sp
    rows = np.repeat(np.arange(nf), np.diff(ptr))
    A = sp.csr_matrix((val, (rows, col)), shape=(nf, nf))
    fn = out["free_nodes"]
    for c in range(3):
        x = out["x"][0, c, fn]
        b = rhs[0, c, fn]
        assert np.linalg.norm(A @ x - b) <= 1e-11 * np.linalg.norm(b)


@pytest.mark.parametrize("name", ["robot", "ragged", "free_block", "one_voxel", "c1"])
@pytest.mark.parametrize("leaf,sep", [(64, 2048), (8, 16)])
def test_host_code_under_sanitizers(sanitized_driver, name, leaf, sep):
    """The host pipeline (mesh, A_s, ordering, factor, sweep plan and the
    bounds-checked sweep replay) runs clean under ASan + UBSan and still solves
    A x = b."""
    sc = CASES[name]()
    o = om.Model(sc)
    rhs = np.random.default_rng(1).standard_normal((1, 3, o.N))
    out = run_driver(sanitized_driver, sc, rhs, leaf, sep)
    b = rhs[0].T.reshape(-1)
    ref = np.zeros(3 * o.N)
    ref[o.free] = o.solve_A(b[o.free])
    got = out["x"][0].T.reshape(-1)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.fixture(scope="module")
def dag_driver(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("dag") / "dag_check")
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-o", out, os.path.join(HERE, "host", "dag_check.cpp"),
           os.path.join(CSRC, "host_mesh.cpp"), os.path.join(CSRC, "factor.cpp")]
    subprocess.run(cmd, check=True)
    return out


DAG_CASES = dict(CASES, block_16=lambda: W.dropped_block(16, 8, 8, steps=1),
                 block_64x32x32=lambda: W.config("c5"))


@pytest.mark.parametrize("name", list(DAG_CASES))
@pytest.mark.parametrize("leaf,sep", [(64, 2048), (8, 16), (512, 2048)])
def test_single_launch_solve_queue(dag_driver, name, leaf, sep):
    """The single-launch solve's queue: every level task in exactly one entry
    in dependency order, and the launch played on the CPU with 1 to 512
    workgroups and random interleavings drains, with every value read after
    it was written and written once (dag_check.cpp)."""
    sc = DAG_CASES[name]()
    if name == "block_64x32x32" and (leaf, sep) != (64, 2048):
        pytest.skip("the benchmark block is checked with the plan it uses")
    with tempfile.TemporaryDirectory() as d:
        fin = os.path.join(d, "in.bin")
        write_input(fin, sc, leaf, sep)
        res = subprocess.run([dag_driver, fin], capture_output=True, text=True)
    print(res.stdout, res.stderr)
    assert res.returncode == 0, res.stderr
