"""Pins for the reference's random streams (SampleStates / SampleControls, Alg. 1).

* Philox4x32-10 against the published Random123 known-answer vectors and
  against rocRAND's independent implementation (its public engine API,
  compiled host-only; no GPU needed).
* The float32 conversion u32 -> [lo, hi] exhaustively over all 2^24 inputs
  against numpy float32 arithmetic.
* The counter layout: branch a = 0 of each query is independent of A.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_2607_03987_amd import workloads as W
from tests.conftest import GOLDEN


def _kat_rows():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            v = [int(t, 16) for t in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat_rows())
def test_philox_known_answers(ctr, key, expect):
    assert list(oracle.philox(ctr, key)) == expect


_ROCRAND_PROBE = r"""
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>
int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
    unsigned long long sub = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
    unsigned long long off = 4ull * ((unsigned long long)c0 | ((unsigned long long)c1 << 32));
    rocrand_device::philox4x32_10_engine e(seed, sub, off);
    uint4 r = e.next4();
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
"""


def test_philox_matches_rocrand_engine(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    src = tmp_path / "probe.cpp"
    src.write_text(_ROCRAND_PROBE)
    exe = tmp_path / "probe"
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O1", str(src), "-o", str(exe)],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    rng = np.random.default_rng(7)
    cases = rng.integers(0, 2**32, size=(200, 6), dtype=np.uint64)
    cases[:, 1] %= 2**30  # the engine's offset is 4*counter in 64 bits
    txt = "\n".join(" ".join(str(int(v)) for v in row) for row in cases) + "\n"
    out = subprocess.run([str(exe)], input=txt, capture_output=True, text=True, check=True).stdout
    got = np.array([[int(t) for t in ln.split()] for ln in out.strip().splitlines()])
    mine = np.array([oracle.philox(r[:4], r[4:]) for r in cases])
    np.testing.assert_array_equal(got, mine)


def test_philox_is_injective_on_sample():
    rng = np.random.default_rng(3)
    ctrs = rng.integers(0, 2**32, size=(4096, 4), dtype=np.uint64)
    outs = {tuple(oracle.philox(c, [11, 22])) for c in ctrs}
    assert len(outs) == len({tuple(c) for c in ctrs})


def test_philox_output_bits_uniform():
    # chi-square on the 256 byte values of 8192 outputs (32768 words)
    words = np.concatenate([oracle.philox([i, 5, 6, 7], [1, 2]) for i in range(8192)])
    counts = np.bincount(words.view(np.uint8), minlength=256)
    expect = counts.sum() / 256
    chi2 = ((counts - expect) ** 2 / expect).sum()
    assert chi2 < 350  # 255 dof: mean 255, sd ~22.6


@pytest.mark.parametrize("lo,hi", [(-1.0, 1.0), (0.0, 10.0), (-np.pi, np.pi), (0.0, 19.62)])
def test_u32_conversion_exhaustive(lo, hi):
    lo32, hi32 = np.float32(lo), np.float32(hi)
    x = (np.arange(1 << 24, dtype=np.uint32) << np.uint32(8)) | np.uint32(0x5A)
    got = oracle.u32_to_range_n(x, lo32, hi32)
    u = (x >> np.uint32(8)).astype(np.float32) * np.float32(2.0 ** -24)
    w = hi32 - lo32
    expect = lo32 + (w * u)
    np.testing.assert_array_equal(got.view(np.uint32), expect.astype(np.float32).view(np.uint32))
    assert got.min() >= lo32 and got.max() <= hi32


def test_sample_state_layout():
    p = W.config_c4()
    cp = oracle.CProblem(p)
    k, it, rnd = 17, 3, 2
    s = oracle.sample_state(cp, k, it, rnd)
    key = [p.seed & 0xFFFFFFFF, p.qid]
    for blk in range(3):
        words = oracle.philox([k, it, rnd, (0 << 16) | blk], key)
        for w in range(4):
            c = 4 * blk + w
            assert s[c] == oracle.u32_to_range(words[w], p.sample_lo[c], p.sample_hi[c])
    assert np.all(s >= p.sample_lo) and np.all(s <= p.sample_hi)


def test_control_branch_zero_independent_of_A():
    p1 = W.config_c1(A=1, B=64)
    p4 = W.config_c1(A=4, B=256)
    c1, c4 = oracle.CProblem(p1), oracle.CProblem(p4)
    for k in range(10):
        np.testing.assert_array_equal(oracle.sample_control(c1, k, 0, 0, 0),
                                      oracle.sample_control(c4, k, 0, 0, 0))
    assert not np.array_equal(oracle.sample_control(c4, 0, 0, 0, 0),
                              oracle.sample_control(c4, 0, 1, 0, 0))
