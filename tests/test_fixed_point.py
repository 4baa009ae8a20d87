"""The fixed-point conversion of the force accumulators, compiled for the
host from the same header the kernels include: defined for every |v| < 2^31
(no out-of-range conversion), exact floor(v 2^32) for v >= 0 and v <= -1,
within 2^8 units of 2^-32 for -1 < v < 0 (where 1 + v is rounded)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def test_to_fix_is_defined_and_exact(tmp_path):
    exe = str(tmp_path / "fixed_check")
    for flags in (["-O0"], ["-O2", "-fsanitize=undefined", "-fno-sanitize-recover=all"]):
        r = subprocess.run(["g++", "-std=c++17", *flags, os.path.join(HERE, "fixed_check.cpp"), "-o", exe],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
        print(r.stdout)
        assert r.returncode == 0, r.stdout + r.stderr
