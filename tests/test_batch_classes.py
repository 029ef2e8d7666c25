"""The batch's binning launch classes (paper_2310_02926_amd/csrc/batch_classes.h)
on the CPU: tests/batch_classes_test.cpp checks the class of a tile's or a
whole grid's LDS at every boundary, hand-made merges of classes too small
to fill the device, and random class sets, asserting that every block is
kept in a class at least its own, that only the largest non-empty class may
stay below the minimum, and that each class's LDS covers its blocks."""
import shutil
import subprocess

import pytest

import os

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "batch_classes_test.cpp")


def _build(tmp_path, sanitize):
    exe = str(tmp_path / ("cls_san" if sanitize else "cls"))
    cmd = ["g++", "-std=c++17", "-O1", "-Wall", "-Wextra", "-Werror", SRC, "-o", exe]
    if sanitize:
        cmd[1:1] = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    p = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    return exe if p.returncode == 0 else None, p.stderr


def test_batch_launch_classes(tmp_path):
    if not shutil.which("g++"):
        pytest.skip("g++ is not available")
    exe, err = _build(tmp_path, sanitize=True)
    if exe is None:  # no sanitizer runtime on this host: build plainly
        exe, err = _build(tmp_path, sanitize=False)
    assert exe is not None, err
    p = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert p.returncode == 0 and p.stdout.strip() == "ok", p.stdout + p.stderr
