"""The 64-bit address split/join of the kernels' buffer descriptors
(paper_1301_5892_amd/csrc/addr.hpp), compiled for the host with g++ and run
on addresses whose low word has bit 31 set.  A sign-extending join of the
same words, which once corrupted descriptor bases, gets those wrong."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_addr_split_join_round_trip(tmp_path):
    exe = tmp_path / "addr_roundtrip"
    src = os.path.join(ROOT, "tests", "addr_roundtrip.cpp")
    inc = os.path.join(ROOT, "paper_1301_5892_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-I", inc, src, "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout
    status, differs = r.stdout.split()
    assert status == "ok"
    assert int(differs) == 4   # the sign-extending join fails the four bit-31 cases
