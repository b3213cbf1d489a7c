"""The host-side packing (validation, exclusion and moving masks, cost, work queues) built
with AddressSanitizer and UndefinedBehaviorSanitizer (g++, host code only) and run over
seeded ligands of the batched workload, each also mutated into invalid forms that must be
refused.  CPU only."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import exs_synth as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2110_11644_amd", "csrc")


def write_vec(f, a, dt):
    a = np.ascontiguousarray(a, dtype=dt)
    f.write(np.int64(a.size).tobytes())
    f.write(a.tobytes())


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_packing_under_sanitizers(tmp_path):
    exe = str(tmp_path / "pack_fuzz")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"),
           "-I" + CSRC, os.path.join(ROOT, "tests", "native", "pack_fuzz.cpp"),
           os.path.join(CSRC, "exs_pack.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    ligs = S.make_ligands("batched", 0, 300) + S.make_ligands("scale", 0, 100)
    b = S.batch_from_ligands(ligs)
    data = str(tmp_path / "ligands.bin")
    with open(data, "wb") as f:
        write_vec(f, b.atom_offset, np.int32)
        for arr in (b.x, b.y, b.z):
            write_vec(f, arr, np.float32)
        write_vec(f, b.type, np.uint8)
        write_vec(f, b.bond_offset, np.int32)
        write_vec(f, b.bond_ij, np.int32)
        write_vec(f, b.rot_offset, np.int32)
        write_vec(f, b.rot_bond, np.int32)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, data], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    packed, refused, tried = (int(w) for w in r.stdout.split()[1::2][:2] + r.stdout.split()[-1:])
    assert packed == len(ligs)
    assert refused == tried > 3 * len(ligs)
