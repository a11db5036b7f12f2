"""Race detection and memory checking of the host code that runs on worker threads.

The domain builder (csrc/domain.cpp) splits the box over up to 16 threads.  It is compiled
here on its own with g++ twice -- AddressSanitizer + UndefinedBehaviorSanitizer, and
ThreadSanitizer -- and driven by tests/c_abi/domain_check.cpp over the three pipe shapes,
closed and open ends, up to a 96x96x160 box.  Each run must be free of sanitizer reports,
and its results must equal those of the library's own build of the same source.

The setup's host-side domain preparation (csrc/host_prep.cpp: argument checks, near-wall
rows and their wall fractions, on up to 16 threads) gets the same two builds, driven by
tests/c_abi/prep_check.cpp over five domains, all three wall rules, shuffled wall entries
and four invalid domains; its rows must equal the ones written out from their definition
with numpy.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = [os.path.join(ROOT, "paper_0907_4863_amd", "csrc", "domain.cpp"),
       os.path.join(ROOT, "tests", "c_abi", "domain_check.cpp")]

CASES = [(0, 1.0, 1.0, 2.0, 0.0, 0.0, 33, 33, 33, 0),
         (1, 1.0, 0.6, 4.0, 0.0, 0.0, 70, 45, 66, 0),
         (2, 0.8, 0.8, 4.0, 0.5, 4.0 / 6.0, 41, 41, 83, 0),
         (0, 1.0, 1.0, 2.0, 0.0, 0.0, 27, 27, 25, 1),
         (1, 1.0, 0.6, 4.0, 0.0, 0.0, 96, 96, 160, 0)]


def _library_lines():
    sa = pytest.importorskip("paper_0907_4863_amd")
    out = []
    for kind, a, b, length, bore, cav, nx, ny, nz, open_ in CASES:
        d = sa.domain_from_shape(kind, a, b, length, nx, ny, nz, bore, cav, bool(open_))
        s = float(np.sum(d.wall_s * (1.0 + d.wall_dir) + 1e-9 * d.wall_node))
        out.append((d.mask.size, int(d.mask.sum()), d.wall_node.size, s))
    return out


@pytest.mark.parametrize("flags", [["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
                                   ["-fsanitize=thread"]], ids=["asan_ubsan", "tsan"])
def test_domain_builder_under_sanitizers(tmp_path, flags):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "domain_check"
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-pthread", *flags,
           f"-I{os.path.join(ROOT, 'include')}", *SRC, "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               TSAN_OPTIONS="halt_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    p = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert p.returncode == 0, p.stderr[-4000:]
    assert "Sanitizer" not in p.stderr and "runtime error" not in p.stderr, p.stderr[-4000:]
    got = [tuple(float(v) for v in ln.split()) for ln in p.stdout.split("\n") if ln.strip()]
    want = _library_lines()
    assert len(got) == len(want)
    for g, w in zip(got, want):
        assert g[:3] == tuple(float(v) for v in w[:3])
        assert abs(g[3] - w[3]) <= 1e-12 * abs(w[3])


# saamg::prepare_domain (csrc/host_prep.cpp: the setup's host-side checks and near-wall rows,
# multithreaded) built alone with the same sanitizers and driven by tests/c_abi/prep_check.cpp
PREP_SRC = [os.path.join(ROOT, "paper_0907_4863_amd", "csrc", "domain.cpp"),
            os.path.join(ROOT, "paper_0907_4863_amd", "csrc", "host_prep.cpp"),
            os.path.join(ROOT, "tests", "c_abi", "prep_check.cpp")]
PREP_CASES = [(0, 1.0, 1.0, 2.0, 0.0, 0.0, 33, 33, 33, 0),
              (2, 0.8, 0.8, 4.0, 0.5, 4.0 / 6.0, 41, 41, 83, 0),
              (0, 1.0, 1.0, 2.0, 0.0, 0.0, 27, 27, 25, 1),
              (1, 1.0, 0.6, 4.0, 0.0, 0.0, 96, 96, 160, 0),
              (1, 1.0, 0.6, 4.0, 0.0, 0.0, 128, 128, 200, 1)]
PREP_ERRORS = ["err duplicate wall entry", "err wall fraction must lie in (1e-12, 1]",
               "err wall entry out of range", "err an unknown lies on a face of the box"]


def _prep_expected():
    """The near-wall rows written out from their definition: every unknown with a wall
    entry whose fraction is below 1 (not for the constant rule) and, with open ends, every
    unknown of box planes 1 and nz-2; fractions 1 except at the cut entries."""
    sa = pytest.importorskip("paper_0907_4863_amd")
    lines = []
    for kind, a, b, length, bore, cav, nx, ny, nz, open_ in PREP_CASES:
        d = sa.domain_from_shape(kind, a, b, length, nx, ny, nz, bore, cav, bool(open_))
        nzb = nz + 2 * open_
        mask = np.asarray(d.mask).reshape(-1)
        nxy = nx * ny
        ends = np.zeros(0, dtype=np.int64)
        if open_:
            ends = np.concatenate([np.nonzero(mask[nxy * k:nxy * (k + 1)])[0] + nxy * k
                                   for k in (1, nzb - 2)]).astype(np.int64)
        node = np.asarray(d.wall_node, dtype=np.int64)
        dirs = np.asarray(d.wall_dir, dtype=np.int64)
        s = np.asarray(d.wall_s, dtype=np.float64)
        per_variant = []
        for variant in (0, 1, 2):
            cut = (s < 1.0) if variant != 0 else np.zeros(s.size, dtype=bool)
            rows = np.union1d(node[cut], ends)
            frac = np.ones((rows.size, 6))
            frac[np.searchsorted(rows, node[cut]), dirs[cut]] = s[cut]
            cs = 0.0
            for v in (frac * (1.0 + np.arange(6))).reshape(-1):
                cs += float(v)
            per_variant.append((rows.size, int(rows.sum()), cs))
        lines += per_variant + [per_variant[2]] + PREP_ERRORS
    return lines


@pytest.mark.parametrize("flags", [["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
                                   ["-fsanitize=thread"]], ids=["asan_ubsan", "tsan"])
def test_domain_preparation_under_sanitizers(tmp_path, flags):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "prep_check"
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-pthread", *flags,
           f"-I{os.path.join(ROOT, 'include')}", *PREP_SRC, "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               TSAN_OPTIONS="halt_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    p = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert p.returncode == 0, p.stderr[-4000:]
    assert "Sanitizer" not in p.stderr and "runtime error" not in p.stderr, p.stderr[-4000:]
    got = [ln for ln in p.stdout.split("\n") if ln.strip()]
    want = _prep_expected()
    assert len(got) == len(want)
    for g, w in zip(got, want):
        if isinstance(w, str):
            assert g == w
        else:
            f = g.split()
            assert f[0] == "ok" and int(f[1]) == w[0] and int(f[2]) == w[1], (g, w)
            assert abs(float(f[3]) - w[2]) <= 1e-13 * max(abs(w[2]), 1.0), (g, w)
