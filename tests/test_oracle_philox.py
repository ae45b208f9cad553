"""Pins of the oracle's counter-based generator (Philox4x32-10 and, from the
same round code, Philox4x64-10; Salmon et al., SC'11)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def test_philox4x64_matches_numpy():
    # numpy's Philox bit generator advances its 256-bit counter before each
    # block, so its first block for counter c is philox4x64(c + 1).
    rng = np.random.default_rng(7)
    for _ in range(20):
        key = [int(x) for x in rng.integers(0, 2**63, size=2, dtype=np.uint64)]
        ctr = [int(x) for x in rng.integers(0, 2**63, size=4, dtype=np.uint64)]
        bg = np.random.Philox(key=np.array(key, np.uint64), counter=np.array(ctr, np.uint64))
        got = [int(x) for x in bg.random_raw(4)]
        ctr1 = list(ctr)
        ctr1[0] += 1
        assert oracle.philox4x64(ctr1, key) == got


@pytest.fixture(scope="module")
def rocrand_kat(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("hipcc / rocRAND headers not available")
    exe = str(tmp_path_factory.mktemp("kat") / "kat")
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O1", "-o", exe,
                           os.path.join(HERE, "helpers", "rocrand_philox_kat.cpp")])
    return exe


def test_philox4x32_matches_rocrand(rocrand_kat):
    rng = np.random.default_rng(11)
    cases, expect = [], []
    for _ in range(64):
        seed = int(rng.integers(0, 2**63))
        c = [int(x) for x in rng.integers(0, 2**32, size=4, dtype=np.uint64)]
        c[1] &= (1 << 29) - 1          # keep 4 * (c0 + c1 << 32) inside 64 bits
        off = 4 * (c[0] + (c[1] << 32))
        sub = c[2] + (c[3] << 32)
        cases.append(f"{seed} {sub} {off}")
        expect.append(oracle.philox4x32(c, [seed & 0xFFFFFFFF, seed >> 32]))
    out = subprocess.run([rocrand_kat], input="\n".join(cases) + "\n", capture_output=True,
                         text=True, check=True).stdout.split("\n")
    for line, e in zip(out, expect):
        assert [int(x) for x in line.split()] == e


def test_philox_zero_vector_words():
    # all-zero counter and key: the block the rocRAND engine above returns
    # for seed 0, subsequence 0, offset 0
    assert oracle.philox4x32([0, 0, 0, 0], [0, 0]) == [0x6627E8D5, 0xE169C58D,
                                                        0xBC57AC4C, 0x9B00DBD8]


def test_words_are_uniform():
    # bits of many blocks: each of the 32 bit positions is set half the time
    words = np.array([oracle.philox4x32([i, 5, 0, 1], [3, 0]) for i in range(4000)],
                     dtype=np.uint64).ravel()
    bits = ((words[:, None] >> np.arange(32, dtype=np.uint64)) & 1).mean(0)
    assert np.all(np.abs(bits - 0.5) < 5 * 0.5 / np.sqrt(words.size))
