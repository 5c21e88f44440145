"""Host check that the adjoint's staged strip record evaluates K as the record
does (Sec. III-C): tests/host_kcut.cpp builds the records of a small cone-beam
scan, converts each as the adjoint's staging does (segment coefficients taken
once, lambda clamped to [d0, dn]) and compares K with the record's own form
(coefficient per term, h clamped to [0, L]) bit for bit, in FP32 and FP64.
It also checks the row-plane split taken from the staged index-scale pairs
against every plane's height range over the strip (Sec. III-C, the planes
wholly below, straddling or wholly above a face), and the adjoint's linear
part of a record (the planes reaching into a voxel from above its bottom
face, summed by parts) against the direct per-plane sum, for voxels holding
0, 1, 2 and 3 or more such planes, and that the zero header of an empty
slot adds exactly zero without reading the table.  Host arithmetic only: no
GPU is used."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _hipcc():
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def test_staged_record_K_equals_record_K():
    if not os.path.exists(_hipcc()):
        pytest.skip("hipcc not found")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "host_kcut")
        cmd = [_hipcc(), "-x", "hip", "--cuda-host-only", "-O2", "-std=c++17",
               "-I" + os.path.join(ROOT, "include"), os.path.join(HERE, "host_kcut.cpp"), "-o", exe]
        r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, r.stderr[-2000:]
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
        print(r.stdout[-2000:])
        assert r.returncode == 0, r.stdout[-2000:]
        lines = {" ".join(l.split()[:2]): l.split() for l in r.stdout.strip().splitlines()}
        lin = lines["linear parts"]
        assert int(lin[3]) > 1000 and lin[5] == "0"
        zero = lines["zero headers"]
        assert int(zero[3]) > 0 and zero[5] == "0"
        splits = lines["splits checked"]
        assert int(splits[2]) > 10000 and splits[4] == "0"
        last = lines["checked " + r.stdout.strip().splitlines()[-1].split()[1]]
        assert int(last[1]) > 100000 and last[3] == "0"
