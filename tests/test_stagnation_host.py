"""The stagnation test of the restart loop (paper_1808_08328_amd/csrc/
stagnation.h) on the CPU: the header is host code without HIP, compiled here
with g++ into a small driver that feeds it residual sequences."""
import shutil
import subprocess

import pytest

HEADER_DIR = __import__("os").path.join(__import__("os").path.dirname(__file__), "..",
                                        "paper_1808_08328_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include "stagnation.h"
// argv: limit ratio r0 r1 ...; prints the index of the first stalled() == true, or -1
int main(int argc, char **argv) {
  dpp::Stagnation s(std::atoi(argv[1]), std::atof(argv[2]));
  for (int i = 3; i < argc; ++i)
    if (s.stalled(std::atof(argv[i]))) { std::printf("%d\n", i - 3); return 0; }
  std::printf("-1\n");
  return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("stag")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    exe = d / "drv"
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", HEADER_DIR, str(src), "-o", str(exe)], check=True)
    return str(exe)


def first_stall(driver, limit, ratio, seq):
    out = subprocess.run([driver, str(limit), repr(ratio)] + [repr(float(v)) for v in seq],
                         capture_output=True, text=True, check=True).stdout
    return int(out)


def test_reducing_cycles_never_stall(driver):
    assert first_stall(driver, 3, 0.999, [1.0, 0.5, 0.2, 0.1, 0.05, 0.01]) == -1


def test_flat_cycles_stall_after_limit(driver):
    # the first call only records the start residual; cycles 1, 2, 3 each stay flat
    assert first_stall(driver, 3, 0.999, [1.0, 1.0, 1.0, 1.0, 1.0]) == 3
    assert first_stall(driver, 1, 0.999, [1.0, 0.9995]) == 1


def test_a_reducing_cycle_resets_the_count(driver):
    seq = [1.0, 0.9999, 0.9998, 0.5, 0.4999, 0.4998, 0.4997]
    assert first_stall(driver, 3, 0.999, seq) == 6


def test_ratio_is_a_strict_bound_and_limit_zero_disables(driver):
    # r = ratio * prev exactly is progress; anything above it is not
    assert first_stall(driver, 1, 0.5, [1.0, 0.5, 0.25]) == -1
    assert first_stall(driver, 1, 0.5, [1.0, 0.6]) == 1
    assert first_stall(driver, 0, 0.999, [1.0] * 10) == -1
