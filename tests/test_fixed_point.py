"""The merge's fixed-point sums (csrc/pp_fixed.h) are exact: compiled for
the host and compared with math.fsum, the correctly rounded sum (Shewchuk),
on cancelling, tiny, huge and random inputs."""
import math
import os
import random
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "fx_check.hip")


@pytest.fixture(scope="module")
def fx_bin(tmp_path_factory):
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("fx") / "fx_check")
    subprocess.check_call(["hipcc", "--offload-arch=gfx950", "-O2", "-std=c++17",
                           f"-I{os.path.join(ROOT, 'paper_2512_12094_amd', 'csrc')}",
                           "-o", out, SRC])
    return out


def run(fx_bin, groups):
    text = "".join(f"{len(g)} " + " ".join(float(v).hex() for v in g) + "\n" for g in groups)
    res = subprocess.run([fx_bin], input=text, capture_output=True, text=True, check=True)
    out = []
    for line in res.stdout.split("\n"):
        if line:
            a, r = line.split()
            out.append((float.fromhex(a), int(r)))
    return out


def test_exact_sums_match_fsum(fx_bin):
    rng = random.Random(7)
    groups = [
        [1e16, 1.0, -1e16],                       # naive FP64 sum gives 0
        [0.1] * 10,
        [1.0, 2.0 ** -52, 2.0 ** -52],            # ties resolved by the tail
        [2.0 ** -52, 1.0, -1.0],
        [3.0, -3.0],
        [-0.0, 0.0],
        [],
        [2.0 ** 53, 1.0, 1.0],
        [-(2.0 ** 53), -1.0],
        [1e15, -1e-10, 3.5e-9, -1e15],
    ]
    for _ in range(300):
        k = rng.randint(1, 60)
        scale = 10.0 ** rng.uniform(-14, 15)
        g = [rng.gauss(0, 1) * scale * 10.0 ** rng.uniform(-6, 0) for _ in range(k)]
        if rng.random() < 0.5:                     # heavy cancellation
            g = g + [-v for v in g[: k // 2]]
            rng.shuffle(g)
        groups.append(g)
    for g, (got, rng_err) in zip(groups, run(fx_bin, groups)):
        assert rng_err == 0
        assert got == math.fsum(g), (g, got, math.fsum(g))


def test_tiny_addends_round_at_the_fixed_point_grid(fx_bin):
    # below 2^(52-104) the addend is rounded to a multiple of 2^-104
    g = [2.0 ** -110, 2.0 ** -110]
    (got, _), = run(fx_bin, [g])
    assert got == 0.0
    (got, _), = run(fx_bin, [[2.0 ** -104 * 3]])
    assert got == 2.0 ** -104 * 3


def test_range_limit(fx_bin):
    (got, r), = run(fx_bin, [[2.0 ** 53]])
    assert r == 0 and got == 2.0 ** 53
    (_, r), = run(fx_bin, [[2.0 ** 54]])
    assert r == 1
    (_, r), = run(fx_bin, [[float("inf")]])
    assert r == 1
