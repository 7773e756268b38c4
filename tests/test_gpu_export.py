"""pp_export_terms returns the set one record per representative, sorted by
key: ascending in the App. E.2 integer (qubit q the base-4 digit of weight
4^q, I, X, Y, Z = 0, 1, 2, 3), the order the oracle's export uses
(Algorithms 2/3 output).  The rows are compared with the oracle's rows
position by position (x/z words bit-exact; coefficients by the rules of
tests/parity.py; strings within the truncation band of eps, which either side
may keep, are dropped from both sequences first), and the order is checked
against the integer computed here from the letters.  Sizes span several
4096-row sort tiles with a ragged last tile; one to four 64-bit words of the
integer (n = 8 to 128); the groups Z_n, D_n, S_n, the torus and none; both
launch paths; FP32 coefficients; an empty set."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2512_12094_amd import workloads as W
from tests.parity import compare_terms, compare_terms_f32, near_threshold

pytestmark = pytest.mark.gpu

DIGIT = {"I": 0, "X": 1, "Y": 2, "Z": 3}


@pytest.fixture(scope="module")
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_12094_amd import _lib
    _lib.lib()
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    return dict(torch=torch, stream=stream, handle=int(stream.cuda_stream),
                alloc=_lib.TorchAllocator(0))


def join(words):
    return sum(int(v) << (64 * w) for w, v in enumerate(words))


def int_value(x, z, n):
    return sum(DIGIT[ch] * 4 ** q for q, ch in enumerate(W.to_letters(x, z, n)))


def keys_of(rows):
    x, z, _ = rows
    return [(join(x[i]), join(z[i])) for i in range(len(x))]


def brickwork(n, steps, theta, eps):
    subs = []
    for _ in range(steps):
        for kind in "XYZ":
            for parity in (0, 1):
                gates = [W.Gate(*W.two_site(kind, b, b + 1), theta)
                         for b in range(parity, n - 1, 2)]
                subs.append(W.SubLayer(gates, eps=eps))
    return W.Program(f"brick{n}", n, "none", W.sum_single(n, "Z"), subs, W.ZERO_STATE,
                     dict(eps=eps))


def prefix(prog, k):
    return W.Program(prog.name + f"[:{k}]", prog.n, prog.group, prog.obs,
                     prog.sublayers[len(prog.sublayers) - k:], prog.bloch, dict(prog.meta))


def sn(n):
    prog = W.heisenberg_all_to_all(n, 1, 0.04, eps=1e-4)
    prog.meta["eps"] = 1e-4
    return prog


CASES = {
    "c1_z8": lambda: W.config1(),
    "c2_z32": lambda: prefix(W.config2(), 36),
    "c2_plain": lambda: W.Program("c2plain", 32, "none", W.config2().obs,
                                  prefix(W.config2(), 8).sublayers, W.config2().bloch,
                                  dict(W.config2().meta)),
    "sn_12": lambda: sn(12),
    "dn_12": lambda: W.xxz_ring(12, 2, 0.25, 1.3, eps=1e-6, group=W.GROUP_DN, name="dn12"),
    "torus_3x3": lambda: W.power_law_xxz_torus(3, 3, 1, 0.1, eps=1e-6),
    "w2_n80": lambda: brickwork(80, 2, 0.2, 1e-4),
    "w2_n100": lambda: brickwork(100, 1, 0.25, 1e-5),
    "w2_n128": lambda: brickwork(128, 1, 0.3, 1e-5),
}


def export_gpu(gpu, prog, program_path, dtype="f64"):
    from paper_2512_12094_amd import _lib as L
    from paper_2512_12094_amd import driver
    ps = driver.PauliSet.from_program(prog, None, gpu["handle"], gpu["alloc"], dtype)
    try:
        if program_path:
            dp = driver.device_program(prog)
            L.pp_batch_run([ps.h], [dp.h], gpu["handle"])
            dp.close()
        else:
            driver.run_layers(ps, driver.heisenberg_layers(prog))
        n_live = ps.num_terms()
        rows = ps.export()
    finally:
        ps.close()
    assert len(rows[2]) == n_live
    return rows


def check_rows(prog, got, want, f32=False):
    n, eps = prog.n, prog.meta.get("eps", 0.0)
    gk, rk = keys_of(got), keys_of(want)
    gd = dict(zip(gk, (float(v) for v in got[2])))
    rd = dict(zip(rk, (float(v) for v in want[2])))
    if f32:
        compare_terms_f32(gd, rd, eps, what=prog.name)
        scale = max([abs(v) for v in rd.values()] + [0.0])
        band = 2.0 ** -21 * scale
    else:
        compare_terms(gd, rd, eps, what=prog.name)
        band = 0.0
    # the order: the same keys in the same positions once the band is dropped
    skip = {k for k, v in gd.items() if near_threshold(v, eps, band)} | \
           {k for k, v in rd.items() if near_threshold(v, eps, band)}
    gs = [k for k in gk if k not in skip]
    rs = [k for k in rk if k not in skip]
    assert gs == rs, f"{prog.name}: export order differs from the oracle's"
    ints = [int_value(x, z, n) for x, z in gk]
    assert all(a < b for a, b in zip(ints, ints[1:])), f"{prog.name}: not ascending"
    return len(gk)


@pytest.mark.parametrize("name", list(CASES))
def test_export_matches_oracle_rows(gpu, name):
    prog = CASES[name]()
    print(f"[case] export {name} n={prog.n} group={prog.group}", flush=True)
    ref = O.run_program(prog, keep_terms=False, keep_rows=True)
    got = export_gpu(gpu, prog, program_path=False)
    rows = check_rows(prog, got, ref.rows)
    assert rows > 0


@pytest.mark.parametrize("name", ["c2_z32", "w2_n80"])
def test_export_program_path(gpu, name):
    """After the device program (layer ops on) the export is the same rows."""
    prog = CASES[name]()
    print(f"[case] export program {name}", flush=True)
    ref = O.run_program(prog, keep_terms=False, keep_rows=True)
    got = export_gpu(gpu, prog, program_path=True)
    assert check_rows(prog, got, ref.rows) > 4096


def test_export_fp32(gpu):
    prog = CASES["c2_z32"]()
    print("[case] export fp32 c2_z32", flush=True)
    ref = O.run_program(prog, keep_terms=False, keep_rows=True)
    got = export_gpu(gpu, prog, program_path=True, dtype="f32")
    check_rows(prog, got, ref.rows, f32=True)


def test_export_spans_tiles_and_empty_set(gpu):
    """A set of several sort tiles exported twice gives the same rows; after
    a truncation that drops every string the export is empty."""
    from paper_2512_12094_amd import _lib as L
    from paper_2512_12094_amd import driver
    prog = CASES["c2_z32"]()
    print("[case] export repeat and empty", flush=True)
    ps = driver.PauliSet.from_program(prog, None, gpu["handle"], gpu["alloc"])
    try:
        driver.run_layers(ps, driver.heisenberg_layers(prog))
        a, b = ps.export(), ps.export()
        assert len(a[2]) > 3 * 4096 and len(a[2]) % 4096 != 0
        for u, v in zip(a, b):
            assert np.array_equal(u, v)
        L.pp_truncate(ps.h, 1e300, -1, 0.0)
        assert ps.num_terms() == 0
        x, z, c = ps.export()
        assert len(c) == 0
    finally:
        ps.close()
