"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): the library's host compressor and container checks
(csv_encode.cpp) and the oracle, built with g++ -fsanitize=address,undefined
into tests/sanitize_driver.cpp, which compresses seeded volumes with both
(brick edges 4..64, one or two tables, rANS and raw nibbles), requires the
same bytes, decodes every brick at every level and checks damaged
containers.  Any sanitizer report fails the test.  (The serving loop and
the pool are host code around HIP calls and need a GPU; they are not
covered here.)"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all", "-g", "-O1"]


@pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None, reason="needs gcc and g++")
def test_host_code_under_asan_and_ubsan(tmp_path):
    orc_o = str(tmp_path / "orc.o")
    enc_o = str(tmp_path / "enc.o")
    exe = str(tmp_path / "sanitize_driver")
    subprocess.run(["gcc", "-c", *SAN, os.path.join(ROOT, "oracle", "csv_oracle.c"), "-o", orc_o], check=True)
    subprocess.run(["g++", "-c", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "paper_2308_16619_amd", "csrc", "csv_encode.cpp"), "-o", enc_o], check=True)
    subprocess.run(["g++", "-std=c++17", *SAN, os.path.join(ROOT, "tests", "sanitize_driver.cpp"), orc_o, enc_o,
                    "-pthread", "-o", exe], check=True)
    vols = {
        "cells": synth.cells(n=64, grid=6, seed=21),
        "voronoi": synth.voronoi_bg(n=64, sites=120, bg=0.3, seed=22),
        "noisy": np.where(np.random.default_rng(23).random((64, 64, 64)) < 0.5,
                          synth.voronoi_bg(n=64, sites=10, seed=24), np.uint32(3)).astype(np.uint32),
    }
    files = []
    for name, v in vols.items():
        p = tmp_path / (name + ".vol")
        with open(p, "wb") as f:
            f.write(np.uint32(v.shape[0]).tobytes())
            f.write(np.ascontiguousarray(v, np.uint32).tobytes())
        files.append(str(p))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe] + files, capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    assert r.stdout.count("every variant agrees") == len(files)
