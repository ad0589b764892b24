"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc, host
code only): every exported routine runs on small inputs and edge cases with no
sanitizer report (any report aborts the run), and its results equal those of the
ordinary build that the other tests load.
"""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

import oracle
from workloads.gen import workload

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]


@pytest.fixture(scope="module")
def san_exe(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    out = str(tmp_path_factory.mktemp("san") / "oracle_san")
    cmd = ["gcc", "-O1", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fexcess-precision=standard",
           "-fopenmp", *SAN, os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(HERE, "oracle_sanitize_main.c"),
           "-o", out, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return out


def _run(exe, tmp_path, pts, eps, mp, threads=4):
    n, d = pts.shape
    src = tmp_path / "in.bin"
    dst = tmp_path / "out.bin"
    with open(src, "wb") as f:
        f.write(struct.pack("<qifi", n, d, np.float32(eps), mp))
        f.write(np.ascontiguousarray(pts, dtype="<f4").tobytes())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1:exitcode=24")
    r = subprocess.run([exe, str(src), str(dst), str(threads)], capture_output=True, text=True, env=env,
                       timeout=300)
    assert r.returncode == 0, f"sanitizer build failed (rc {r.returncode}):\n{r.stderr[-4000:]}"
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    buf = open(dst, "rb").read()
    off = 0
    res = []
    for _ in range(2):
        k = struct.unpack_from("<q", buf, off)[0]
        off += 8
        lab = np.frombuffer(buf, "<i4", n, off)
        off += 4 * n
        core = np.frombuffer(buf, np.uint8, n, off)
        off += n
        cnt = np.frombuffer(buf, "<i4", n, off)
        off += 4 * n
        bad = struct.unpack_from("<q", buf, off)[0]
        off += 8
        res.append((k, lab, core, cnt, bad))
    nb0 = struct.unpack_from("<q", buf, off)[0]
    return res, nb0


def _cases():
    rng = np.random.default_rng(77)
    yield "c1_blobs", workload("c1_blobs2d_16k").points, 0.01, 5
    yield "c3_slice", workload("c3_dense3d_8m", 1 / 2048).points, 0.002, 10
    yield "one_point", np.zeros((1, 3), np.float32), 0.5, 1
    yield "duplicates", np.full((300, 2), 0.25, np.float32), 0.1, 7
    yield "pairs_at_eps", np.array([[0, 0, 0], [0.5, 0, 0], [3, 0, 0], [3.5, 0, 0]], np.float32), 0.5, 2
    yield "wide_2d", (rng.uniform(-1e3, 1e3, size=(2000, 2))).astype(np.float32), 30.0, 3
    yield "line_3d", np.stack([np.arange(500) * 0.25, np.zeros(500), np.zeros(500)], 1).astype(np.float32), 0.25, 3


@pytest.mark.parametrize("case", list(range(7)))
def test_sanitized_oracle_matches_plain_build(san_exe, tmp_path, case):
    name, pts, eps, mp = list(_cases())[case]
    (rb, rg), nb0 = _run(san_exe, tmp_path, pts, eps, mp)
    labels, core, k = oracle.dbscan(pts, eps, mp)
    for kk, lab, co, cnt, bad in (rb, rg):
        assert kk == k, name
        assert np.array_equal(lab, labels), name
        assert np.array_equal(co.astype(bool), core), name
        assert np.array_equal(cnt, oracle.neighbor_counts(pts, eps)), name
        assert bad == 0, name
    assert nb0 == len(oracle.neighbors_of(pts, eps, 0)), name
