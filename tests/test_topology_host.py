"""Host topology builder (no GPU): built with g++ under AddressSanitizer and
UndefinedBehaviorSanitizer and run on valid meshes (single tet, jittered cube,
notched beam, coarse ellipsoid) and on invalid ones (node id out of range,
repeated node, flat tet): the pattern, its compact halves and the
contribution slots are consistent, invalid meshes are rejected, and the
sanitizers report nothing."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2103_14870_amd import meshgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def write_mesh(path, X, T):
    with open(path, "wb") as f:
        np.array([X.shape[0], T.shape[0]], np.int32).tofile(f)
        np.ascontiguousarray(X, np.float64).tofile(f)
        np.ascontiguousarray(T, np.int32).tofile(f)


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("topo") / "topo_check")
    csrc = os.path.join(ROOT, "paper_2103_14870_amd", "csrc")
    subprocess.run([gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", "-I", csrc, "-o", exe, os.path.join(ROOT, "tests", "topo_check.cpp"),
                    os.path.join(csrc, "topo.cpp")], check=True, capture_output=True)
    return exe


def run(exe, path):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    return subprocess.run([exe, path], capture_output=True, text=True, env=env, timeout=120)


def test_valid_meshes(checker, tmp_path):
    tet = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
    h = 0.08
    grid = (int(math.ceil(2.1 / h)) | 1, int(math.ceil(1.1 / h)) | 1, int(math.ceil(1.1 / h)) | 1)
    cases = {"tet": (tet, np.array([[0, 1, 3, 2]])),
             "cube": meshgen.tiny_cube(3, h=0.1, jitter_frac=0.05, seed=1),
             "beam": meshgen.notched_beam(16, 4, 4, h=0.01, notch_cells=1),
             "ellipsoid": meshgen.ellipsoid(h=h, grid=grid)}
    for name, c in cases.items():
        X, T = c if isinstance(c, tuple) else (c.X, c.tets)
        path = str(tmp_path / f"{name}.bin")
        write_mesh(path, X, T)
        r = run(checker, path)
        assert r.returncode == 0 and r.stdout.strip() == "bad 0", (name, r.stdout, r.stderr[-2000:])
        assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr


def test_invalid_meshes_are_rejected(checker, tmp_path):
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
    flat = X.copy()
    flat[3] = [0.5, 0.5, 0.0]
    cases = {"id": (X, [[0, 1, 3, 7]], "outside"), "repeat": (X, [[0, 1, 1, 2]], "repeats"),
             "flat": (flat, [[0, 1, 3, 2]], "zero volume")}
    for name, (Xc, T, msg) in cases.items():
        path = str(tmp_path / f"{name}.bin")
        write_mesh(path, Xc, np.array(T))
        r = run(checker, path)
        assert r.returncode == 1 and r.stdout.startswith("err") and msg in r.stdout, (name, r.stdout, r.stderr[-2000:])
        assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr


def test_nonlocal_support_matches_the_oracle(checker, tmp_path):
    """The library's support of Eq. 20 (uniform-grid search, host side) equals
    the oracle's (k-d tree query) entry for entry: the same neighbour sets in
    ascending order and the same normalised weights; a radius below the
    centroid spacing leaves each tet alone; a non-positive radius is refused."""
    from oracle import gfem_oracle as O

    prob = meshgen.cube_block(5, 4, 3, h=0.1, jitter_frac=0.08, seed=3)
    path = str(tmp_path / "cube.bin")
    write_mesh(path, prob.X, prob.tets)
    for radius in (1e-4, 0.17, 0.31):
        out = str(tmp_path / "support.bin")
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
        r = subprocess.run([checker, path, repr(radius), out], capture_output=True, text=True, env=env, timeout=120)
        assert r.returncode == 0 and r.stdout.strip() == "bad 0", r.stdout + r.stderr[-2000:]
        raw = open(out, "rb").read()
        m, ne = np.frombuffer(raw[:16], np.int64)
        ptr = np.frombuffer(raw[16:16 + 8 * (m + 1)], np.int64)
        idx = np.frombuffer(raw[16 + 8 * (m + 1):16 + 8 * (m + 1) + 4 * ne], np.int32)
        w = np.frombuffer(raw[16 + 8 * (m + 1) + 4 * ne:], np.float64)
        mesh = O.setup(prob.X, prob.tets, dict(prob.params, damage_radius=radius))
        optr, oidx, ow = mesh.nonlocal_support
        assert np.array_equal(ptr, optr) and np.array_equal(idx, oidx)
        np.testing.assert_allclose(w, ow, rtol=1e-13, atol=1e-15)
        if radius < 0.01:
            assert np.array_equal(np.diff(ptr), np.ones(m))
    bad = subprocess.run([checker, path, "0", str(tmp_path / "x.bin")], capture_output=True, text=True, timeout=60)
    assert bad.returncode == 1 and "radius" in bad.stdout


def test_rcm_renumbering_restores_a_narrow_band(checker, tmp_path):
    """A notched beam whose node ids are randomly permuted has a band of the
    order of n; reverse Cuthill-McKee renumbering brings it back within
    twice the band of the generator's own lexicographic order (and keeps the
    pattern, slot maps and the caller-to-internal mapping consistent)."""
    prob = meshgen.notched_beam(24, 6, 6, h=0.01, notch_cells=1)
    X, T = prob.X, prob.tets
    n = X.shape[0]
    e = meshgen.unique_edges(T)
    band0 = int((e[:, 1] - e[:, 0]).max())
    perm = np.random.default_rng(5).permutation(n)          # new id of each old node
    Xp = np.empty_like(X)
    Xp[perm] = X
    Tp = perm[T].astype(np.int32)
    ep = meshgen.unique_edges(Tp)
    band_p = int((ep[:, 1] - ep[:, 0]).max())
    path = str(tmp_path / "perm.bin")
    write_mesh(path, Xp, Tp)
    r = subprocess.run(
        [checker, path, "--rcm"], capture_output=True, text=True, timeout=120,
        env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
    out = r.stdout.split()
    assert r.returncode == 0 and out[:2] == ["bad", "0"], r.stdout + r.stderr[-2000:]
    band_rcm = int(out[3])
    assert band_p > 0.5 * n and band_rcm <= 2 * band0, (band0, band_p, band_rcm)
