"""The file readers (host C++, include/fwh_io.h) built with AddressSanitizer and
UndefinedBehaviorSanitizer into a small driver and run over valid, truncated,
corrupted and random files: every call must return a documented code without a
memory error.  CPU only; skipped if the host compiler has no sanitizer runtime."""
import os
import random
import shutil
import struct
import subprocess

import numpy as np
import pytest

from paper_2312_16263_amd import fileio

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2312_16263_amd", "csrc", "fwh_io.cpp")
GOLDEN = os.path.join(ROOT, "tests", "golden", "opencfd_case")

DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>
#include "fwh_io.h"

// usage: driver <kind> <path|dir>; prints the return code
int main(int argc, char **argv) {
    const char *kind = argv[1], *path = argv[2];
    int rc = 0;
    if (!strcmp(kind, "control")) {
        int32_t n = 0;
        rc = fwh_io_control_read(path, nullptr, 0, &n);
        if (rc == 0) {
            std::vector<fwh_io_kv> kv(n > 0 ? n : 1);
            rc = fwh_io_control_read(path, kv.data(), n, &n);
        }
    } else if (!strcmp(kind, "geometry")) {
        int64_t nf = 0, np = 0;
        rc = fwh_io_geometry_read(path, &nf, &np, nullptr, nullptr, nullptr, nullptr, 0, 0);
        if (rc == 0) {
            std::vector<int64_t> d(3 * nf);
            std::vector<double> y(3 * np + 1), n(3 * np + 1), s(np + 1);
            rc = fwh_io_geometry_read(path, &nf, &np, d.data(), y.data(), n.data(), s.data(), nf, np);
        }
    } else if (!strcmp(kind, "observers")) {
        int64_t no = 0;
        rc = fwh_io_observers_read(path, &no, nullptr, 0);
        if (rc == 0) {
            std::vector<double> x(3 * no + 1);
            rc = fwh_io_observers_read(path, &no, x.data(), no);
        }
    } else {  // frames: dir with FWH-00000000.dat .. of Faces [2,1,1],[1,1,3]
        const int64_t dims[6] = {2, 1, 1, 1, 1, 3};
        const int fmt = !strcmp(kind, "ascii") ? 1 : 0;
        const int64_t N = 2, P = 5;
        std::vector<double> rho(N * P), u(3 * N * P), pp(N * P);
        rc = fwh_io_frames_read(path, 0, 1, N, fmt, 2, dims, 0, rho.data(), u.data(), pp.data(), 2);
        std::vector<float> r32(N * P), u32(3 * N * P), p32(N * P);
        const int rc32 = fwh_io_frames_read(path, 0, 1, N, fmt, 2, dims, 1, r32.data(), u32.data(), p32.data(), 3);
        if (rc32 != rc) rc = 99;
    }
    printf("%d\n", rc);
    return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    d = tmp_path_factory.mktemp("asan")
    drv = d / "driver.cpp"
    drv.write_text(DRIVER)
    exe = d / "driver"
    cmd = [gxx, "-std=c++17", "-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "include"), str(drv), SRC, "-o", str(exe), "-pthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("sanitizer build unavailable: " + r.stderr[-300:])
    return str(exe)


def _run(exe, kind, path):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, kind, path], capture_output=True, text=True, env=env, timeout=60)
    assert r.returncode == 0, (kind, path, r.stderr[-2000:])
    assert "runtime error" not in r.stderr, r.stderr[-2000:]
    return int(r.stdout.strip())


def _frames(d, fmt, blobs):
    for k, b in enumerate(blobs):
        with open(os.path.join(d, "FWH-%08d.dat" % k), "wb") as f:
            f.write(b)


def test_sanitized_readers(driver, tmp_path):
    rng = random.Random(11)
    ok, bad = fileio.FWH_IO_OK, fileio.FWH_IO_EFORMAT
    # valid inputs
    assert _run(driver, "control", os.path.join(GOLDEN, "control.fwh")) == ok
    assert _run(driver, "geometry", os.path.join(GOLDEN, "FWH_Surface_Geo.dat")) == ok
    assert _run(driver, "observers", os.path.join(GOLDEN, "observers.dat")) == ok
    dims = np.array([[2, 1, 1], [1, 1, 3]], dtype=np.int64)
    v = np.arange(25, dtype=np.float64).reshape(5, 5)
    good = {}
    for fmt, kind in ((fileio.BINARY, "binary"), (fileio.ASCII, "ascii")):
        d = tmp_path / kind
        d.mkdir()
        for k in range(2):
            fileio.write_frame(fileio.frame_path(str(d), k), fmt, dims, v[0], v[1:4], v[4])
        good[kind] = open(fileio.frame_path(str(d), 0), "rb").read()
        assert _run(driver, kind, str(d)) == ok
    # truncated and corrupted frames, both formats
    for kind, blob in good.items():
        d = tmp_path / (kind + "_bad")
        d.mkdir()
        cuts = sorted(set(rng.randrange(len(blob)) for _ in range(12)) | {0, 1, len(blob) - 1})
        for n in cuts:
            _frames(str(d), kind, [blob, blob[:n]])
            assert _run(driver, kind, str(d)) in (bad, ok if kind == "ascii" else bad)
        for _ in range(12):
            b = bytearray(blob)
            for _ in range(3):
                b[rng.randrange(len(b))] = rng.randrange(256)
            _frames(str(d), kind, [blob, bytes(b)])
            assert _run(driver, kind, str(d)) in (ok, bad, fileio.FWH_IO_ESIZE)
        if kind == "binary":  # a length word claiming 4 GiB
            b = bytearray(blob)
            b[20:24] = struct.pack("<I", 0xFFFFFFF0)
            _frames(str(d), kind, [blob, bytes(b)])
            assert _run(driver, kind, str(d)) == bad
    # random and adversarial text for the text readers
    samples = ["", "\n\n", "variables\n", "variables\n1\n", "variables\n-3\n", "variables\n1\n1 1 1\n" + "1 " * 6,
               "&g a = '" + "x" * 500 + "'\n/", "&g " + "a=1," * 1000 + "/", "&g a = 'unterminated", "&" * 300,
               "1e999 2 3\n", "1 2 " + "9" * 5000 + "\n", "nan inf -inf\n", "\x00\x01\x02", "! only a comment\n"]
    for _ in range(20):
        samples.append("".join(rng.choice("&/=,'! \n0123456789.eEdD-+abcxyz") for _ in range(rng.randrange(1, 400))))
    for i, text in enumerate(samples):
        p = tmp_path / ("t%d.txt" % i)
        p.write_bytes(text.encode("latin-1"))
        for kind in ("control", "geometry", "observers"):
            assert _run(driver, kind, str(p)) in (ok, bad, fileio.FWH_IO_ESIZE)
