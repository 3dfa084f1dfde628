"""CPU-side checks of the library: it loads, exports every entry point that
include/mvn.h declares, sizes buffers without a device, and its device
arithmetic (compiled for the host from the same header) matches SciPy."""
import ctypes
import os
import re
import shutil
import subprocess

import numpy as np
import pytest
import scipy.special as sp

import paper_2405_14892_amd as mvn
from paper_2405_14892_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "mvn.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(mvn_\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    h = ctypes.CDLL(_lib.LIB_PATH)
    names = _declared_symbols()
    assert len(names) >= 6
    for name in names:
        assert hasattr(h, name), name
        assert name in _lib.SIGNATURES, name
    assert _lib.lib().mvn_version() >= 100


def test_size_queries_and_host_validation_need_no_device():
    opts = mvn.options(tile=128)
    fb = mvn.mvn_factor_bytes(400, opts)
    assert fb >= 512 * 512 * 8
    ws = mvn.mvn_prob_workspace_bytes(400, 10_000, 10, opts)
    # per-sample log-products + one 512 x 128 scratch block per workgroup
    assert ws >= 10_000 * 10 * 8 + 256 * 512 * 128 * 8
    with pytest.raises(mvn.MvnError) as e:
        mvn.mvn_factor_bytes(0, opts)
    assert e.value.code == -1
    with pytest.raises(mvn.MvnError) as e:
        mvn.mvn_prob_workspace_bytes(10, 5, 0, opts)
    assert e.value.code == -3
    h = _lib.lib()
    out = _lib.MvnFactor()
    code = h.mvn_cholesky(0, None, 0, None, None, ctypes.byref(opts), None, 0, None, 0,
                          ctypes.byref(out), None)
    assert code == -1 and b"n must be" in h.mvn_last_error()


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("h") / "math_harness")
    src = os.path.join(ROOT, "tests", "host", "math_harness.cpp")
    subprocess.run([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O2", "-o", exe, src], check=True,
                   capture_output=True)
    return exe


def _run(exe, lines):
    out = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True,
                         check=True).stdout
    return [l for l in out.split("\n") if l]


def test_as241_inverse_normal_matches_scipy(harness):
    ps = np.concatenate([np.logspace(-300, -1, 2000), np.linspace(0.01, 0.5, 1000)])
    got = np.array([float(v) for v in _run(harness, [f"ninv {float(p)!r}" for p in ps])])
    rel = np.abs(got - sp.ndtri(ps)) / np.abs(sp.ndtri(ps)).clip(1e-300)
    assert rel.max() < 2e-15


def test_as241_table_form_equals_select_form(harness):
    """The sweeps read the AS 241 coefficients from an LDS copy of the table;
    the result must be the select form's, bit for bit, in all three ranges."""
    ps = np.concatenate([np.logspace(-300, -0.31, 1500), np.linspace(0.07, 0.5, 500),
                         [1e-300, 0.075, 0.0750001, 0.5, np.exp(-25.0), np.exp(-25.0) * 1.0000001]])
    got = _run(harness, [f"ninvtab {float(p)!r}" for p in ps])
    assert len(got) == len(ps) and all(v == "1" for v in got)


def test_conditioning_step_matches_oracle(harness):
    from oracle import sov
    rng = np.random.default_rng(0)
    al = np.concatenate([rng.normal(0, 3, 1500), rng.uniform(-60, 60, 500), [-np.inf] * 100])
    be = al + np.abs(rng.normal(0, 3, al.size))
    be[:150] = np.inf
    be[np.isinf(al)] = rng.normal(0, 10, 100)
    w = rng.uniform(size=al.size)
    res = _run(harness, [f"cond {float(a)!r} {float(b)!r} {float(x)!r}" for a, b, x in zip(al, be, w)])
    gy = np.array([float(r.split()[0]) for r in res])
    gl = np.array([float(r.split()[1]) for r in res])
    oy, ol = sov.condition(al, be, w)
    assert np.max(np.abs(gy - oy)) < 1e-11
    assert np.max(np.abs(gl - ol) / np.maximum(1, np.abs(ol))) < 1e-12


def test_splitmix64_matches_published_outputs(harness):
    got = [int(v) for v in _run(harness, ["sm 0 0", "sm 0 1", "sm 0 2"])]
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_counter_normals_match_oracle_draws(harness):
    """The device's normal draws (AS 241 on the SplitMix64 uniform) against
    the oracle's (scipy's inverse normal on the same uniform), over sites
    and samples of a 7-site field, tails included."""
    from oracle import mc
    n, cols, seed = 7, np.array([0, 1, 5, 1000, 123456]), 99
    ref = mc.normals(seed, n, cols)
    lines = [f"mcn {seed} {int(j) * n + i}" for j in cols for i in range(n)]
    got = np.array([float(v) for v in _run(harness, lines)]).reshape(len(cols), n).T
    np.testing.assert_allclose(got, ref, rtol=2e-15, atol=1e-15)
    # deep tail: the smallest and largest uniforms the stream can give
    z = [float(v) for v in _run(harness, ["ninv 5.551115123125783e-17"])]
    assert abs(z[0] - sp.ndtri(2.0 ** -54)) < 1e-13


def test_matern_general_nu_matches_oracle_and_high_precision(harness):
    """The device covariance (trapezoidal rule on the integral form of
    K_nu, compiled for the host) against the oracle (scipy's K_nu, about
    1e-13) and 40-digit values, at smoothness values off the closed forms,
    distances from 1e-7 to 60 ranges; the closed forms at nu = 1/2, 3/2, 5/2."""
    import oracle
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 40
    beta = 0.05
    hs = np.concatenate([[1e-7, 1e-5], np.logspace(-3.5, np.log10(3.0), 25)])
    for nu in (0.05, 0.3, 0.7, 1.0, 1.2, 1.43391, 2.0, 2.5, 3.3, 7.0, 0.5, 1.5):
        lines = [f"matern 1.3 {beta!r} {nu!r} {float(h)!r}" for h in hs]
        got = np.array([float(v) for v in _run(harness, lines)])
        ref = oracle.matern(hs, 1.3, beta, nu)
        ok = ref > 1e-250
        np.testing.assert_allclose(got[ok], ref[ok], rtol=5e-13, atol=0, err_msg=f"nu={nu}")
        for h, g in list(zip(hs, got))[::4]:
            z = mp.mpf(float(h)) / mp.mpf(beta)
            hp = 1.3 * z ** nu * mp.besselk(nu, z) / (mp.mpf(2) ** (nu - 1) * mp.gamma(nu))
            if float(hp) > 1e-250:
                assert abs(g / float(hp) - 1) < 1e-13, (nu, h)
    # h = 0 gives sigma^2 for every nu
    assert [float(v) for v in _run(harness, ["matern 1.3 0.05 1.43391 0", "matern 1.3 0.05 0.3 0"])] == [1.3, 1.3]


def test_mc_workspace_query_needs_no_device():
    n, M = 1000, 50_000
    ws = mvn.mvn_mc_prefix_workspace_bytes(n, M)
    # per-workgroup Z scratch (1024 x 64 doubles for n = 1000) for min(chunks, 512) workgroups
    # (128-row blocks, two per CU; 64-row blocks: four per CU)
    assert ws >= min((M + 63) // 64, 256 * 2) * 1024 * 64 * 8 + (n + 1) * 8
    ws64 = mvn.mvn_mc_prefix_workspace_bytes(n, M, mvn.options(sweep_rows=64))
    assert ws64 >= min((M + 63) // 64, 256 * 4) * 1024 * 64 * 8 + (n + 1) * 8
    assert mvn.mvn_mc_prefix_workspace_bytes(n, 64) >= 1024 * 64 * 8
    with pytest.raises(mvn.MvnError) as e:
        mvn.mvn_mc_prefix_workspace_bytes(0, 10)
    assert e.value.code == -1


def test_ctypes_structs_match_the_c_header(tmp_path):
    """sizeof / offsetof of the public structs, from the C compiler, equal the
    ctypes mirrors the binding passes by reference."""
    fields = {"mvn_options": _lib.MvnOptions, "mvn_factor": _lib.MvnFactor, "mvn_matern": _lib.MvnMatern}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "mvn.h"', "int main(void) {"]
    for cname, cls in fields.items():
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = str(tmp_path / "layout")
    subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"), "-I", "/opt/rocm/include",
                    str(src), "-o", exe], check=True, capture_output=True)
    out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {(a, b): int(c) for a, b, c in (l.split() for l in out if l)}
    for cname, cls in fields.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)


def test_tlr_size_queries_and_option_checks():
    opts = mvn.options(tile=256, tlr_eps=1e-6, max_rank=100)
    n, m, rs = 1000, 256, 112
    nt = 4
    fb = mvn.mvn_factor_bytes(n, opts)
    tiles = nt * (nt + 1) // 2 * m * m * 8
    panels = nt * (nt - 1) // 2
    assert fb >= tiles + panels * m * rs * 8 * 2 + 128 * m * 8 + panels * 4
    assert fb < tiles + panels * m * rs * 8 * 2 + 128 * m * 8 + 8192
    ws = mvn.mvn_cholesky_workspace_bytes(n, opts)
    assert ws >= panels * (rs * rs + m * rs) * 8
    assert mvn.mvn_cholesky_workspace_bytes(n, mvn.options(tile=256)) == 0
    pw = mvn.mvn_prob_workspace_bytes(n, 1000, 2, opts)
    assert pw >= 2000 * 8 + 32 * (nt * m * 64 + (nt - 1) * rs * 64) * 8
    for bad in (dict(tile=200), dict(tile=2048), dict(max_rank=0), dict(max_rank=300),
                dict(precision=mvn.MVN_FP32)):
        kw = dict(tile=256, tlr_eps=1e-6, max_rank=100)
        kw.update(bad)
        with pytest.raises(mvn.MvnError) as e:
            mvn.mvn_factor_bytes(n, mvn.options(**kw))
        assert e.value.code == -2, bad
    # the batched entry point takes dense factors only
    h = _lib.lib()
    plan = ctypes.create_string_buffer(4096)
    sizes = (ctypes.c_int * 1)(10)
    code = h.mvn_prob_batch(1, sizes, plan, ctypes.c_void_p(8), ctypes.c_void_p(8),
                            ctypes.byref(_lib.MvnMatern(1.0, 0.1, 0.5, 0.0)), ctypes.c_void_p(8),
                            ctypes.c_void_p(8), None, 10, 1, 1, ctypes.byref(opts), None, 0, None, 0, None,
                            None, None)
    assert code == -13 and b"dense" in h.mvn_last_error()


def test_tlr_sweep_form_choice_in_the_size_query():
    """TLR factors take sweep_rows 0 (= 64), 64, 128 or 256 (the four-wave
    form: 256 columns per workgroup, Y and Z slices four times as wide, on
    request only); dense factors refuse 256."""
    n = 1000
    base = dict(tile=256, tlr_eps=1e-6, max_rank=100)
    size = lambda N, S, rows: mvn.mvn_prob_workspace_bytes(n, N, S, mvn.options(sweep_rows=rows, **base))
    # (the slices differ in total width where the chunk counts do not fill
    # the workgroup caps the same way: 625 chunks of 64 against 157 of 256,
    # and 1024 capped chunks of 64 against 391 of 256)
    for N, S in ((1000, 2), (20_000, 2), (65536, 1), (10_000, 10)):
        assert size(N, S, 0) == size(N, S, 64)
    assert size(20_000, 2, 256) != size(20_000, 2, 64)
    assert size(10_000, 10, 256) != size(10_000, 10, 64)
    for bad in (32, 96, 512):
        with pytest.raises(mvn.MvnError):
            size(1000, 2, bad)
    with pytest.raises(mvn.MvnError):
        mvn.mvn_prob_workspace_bytes(n, 1000, 2, mvn.options(tile=64, sweep_rows=256))


def test_fp32_inverse_normal_within_single_precision(harness):
    """PPND7 in FP32 (the reduced-precision modes' central Phi^-1) against
    SciPy: absolute error below 3e-7 (1 + |y|) from p = 1e-33 to 1/2."""
    ps = np.concatenate([np.logspace(-33, -1, 2000), np.linspace(0.01, 0.5, 1000)])
    got = np.array([float(v) for v in _run(harness, [f"ninv32 {float(p)!r}" for p in ps])])
    ref = sp.ndtri(ps.astype(np.float32).astype(np.float64))
    assert np.max(np.abs(got - ref) / (1 + np.abs(ref))) < 3e-7


def test_mixed_conditioning_step_close_to_oracle(harness):
    """The reduced-precision step (FP32 central Phi / Phi^-1, FP64 tails)
    against the oracle's FP64 step: y within 1e-5 (1 + |y|), log d within
    1e-5, on the same inputs as the FP64 check (wide, narrow, deep and
    one-sided intervals)."""
    from oracle import sov
    rng = np.random.default_rng(0)
    al = np.concatenate([rng.normal(0, 3, 1500), rng.uniform(-60, 60, 500), [-np.inf] * 100])
    be = al + np.abs(rng.normal(0, 3, al.size))
    be[:150] = np.inf
    be[np.isinf(al)] = rng.normal(0, 10, 100)
    w = rng.uniform(size=al.size)
    res = _run(harness, [f"condmix {float(a)!r} {float(b)!r} {float(x)!r}" for a, b, x in zip(al, be, w)])
    gy = np.array([float(r.split()[0]) for r in res])
    gl = np.array([float(r.split()[1]) for r in res])
    oy, ol = sov.condition(al, be, w)
    assert np.max(np.abs(gy - oy) / (1 + np.abs(oy))) < 1e-5
    fin = np.isfinite(ol)
    assert np.array_equal(fin, np.isfinite(gl))
    assert np.max(np.abs(gl[fin] - ol[fin])) < 1e-5


@pytest.fixture(scope="module")
def tables_exe(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("t") / "tlr_tables_dump")
    src = os.path.join(ROOT, "tests", "host", "tlr_tables_dump.cpp")
    subprocess.run(["g++", "-O1", "-std=c++17", "-o", exe, src], check=True)
    return exe


def _tables(exe, nt, rs, ranks):
    txt = f"{nt} {rs}\n" + " ".join(str(int(r)) for r in ranks) + "\n"
    out = subprocess.run([exe], input=txt, capture_output=True, text=True, check=True).stdout
    res = {}
    for line in out.strip().split("\n"):
        name, *vals = line.split()
        res[name] = np.array([int(v) for v in vals], dtype=np.int64)
    return res


@pytest.mark.parametrize("nt,rs,seed", [(1, 16, 0), (2, 16, 1), (7, 32, 2), (12, 48, 3)])
def test_tlr_sweep_tables(tables_exe, nt, rs, seed):
    """The TLR sweep's packing: V' rows stacked by tile column in order of the
    tile-row, U columns of a tile-row packed in order of the tile column and
    padded to 16, and the map from stacked rows to packed rows a bijection
    onto the unpadded rows (every product lands where its tile-row reads it)."""
    rng = np.random.default_rng(seed)
    npairs = nt * (nt - 1) // 2
    ranks = rng.integers(0, rs + 1, npairs)
    ranks[rng.random(npairs) < 0.3] = 0
    ranks[rng.random(npairs) < 0.2] *= -1  # capped tiles carry a negative rank
    if npairs:
        ranks[0] = -(2 ** 31)  # a garbage rank is clipped to the stride
    T = _tables(tables_exe, nt, rs, ranks)
    k = np.minimum(np.abs(ranks.astype(np.int64)), rs)
    pair = lambda i, j: i * (i - 1) // 2 + j
    if npairs:
        assert np.array_equal(T["k"], k)
    assert T["ksum"][0] == k.sum()
    # stacked V' rows: column j holds pairs (j+1, j), (j+2, j), ... in order
    row = 0
    for j in range(nt):
        assert T["zcol"][j] == row
        for i in range(j + 1, nt):
            assert T["vrow0"][pair(i, j)] == row
            row += k[pair(i, j)]
    assert T["zcol"][nt] == row
    # packed K of tile-row i: pairs (i, 0), (i, 1), ... then zero padding to 16
    for i in range(nt):
        c = 0
        for j in range(i):
            assert T["ucol0"][pair(i, j)] == c
            c += k[pair(i, j)]
        assert T["kval"][i] == c
        width = T["kpad0"][i + 1] - T["kpad0"][i]
        assert width % 16 == 0 and c <= width < c + 16
    assert T["kpad0"][0] == 0
    # zdst: stacked row -> packed row, a bijection onto the unpadded rows
    want = []
    for i in range(nt):
        want.extend(range(T["kpad0"][i], T["kpad0"][i] + T["kval"][i]))
    assert sorted(T["zdst"].tolist()) == want
    for i in range(1, nt):
        for j in range(i):
            p = pair(i, j)
            for q in range(k[p]):
                assert T["zdst"][T["vrow0"][p] + q] == T["kpad0"][i] + T["ucol0"][p] + q


def test_permuted_cholesky_and_posterior_host_validation():
    """Argument checks of mvn_cholesky_permuted and mvn_posterior, which all
    run before any device call (argument positions as returned codes).  The
    index arrays themselves are device arrays, checked on the device."""
    h = _lib.lib()
    opts = mvn.options(tile=64)
    out = _lib.MvnFactor()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    n = 4
    ok = fake
    code = h.mvn_cholesky_permuted(n, fake, n, None, ctypes.byref(opts), fake, 1 << 20, fake, 1 << 20,
                                   ctypes.byref(out), None)
    assert code == -4
    code = h.mvn_cholesky_permuted(n, fake, n, ok, ctypes.byref(opts), None, 1 << 20, fake, 1 << 20,
                                   ctypes.byref(out), None)
    assert code == -6
    code = h.mvn_cholesky_permuted(n, fake, n, ok, ctypes.byref(opts), fake, 8, fake, 1 << 20, ctypes.byref(out), None)
    assert code == -7
    code = h.mvn_cholesky_permuted(n, fake, n, ok, ctypes.byref(opts), fake, 1 << 20, fake, 0, ctypes.byref(out), None)
    assert code == -9
    code = h.mvn_cholesky_permuted(n, fake, 2, ok, ctypes.byref(opts), fake, 1 << 20, fake, 1 << 20,
                                   ctypes.byref(out), None)
    assert code == -3
    km = _lib.MvnMatern(1.0, 0.1, 0.5, 0.0)
    obs = fake
    mu_p, ld_p = ctypes.c_void_p(0), ctypes.c_int(0)
    args = lambda o, noise, wsb: (10, fake, None, 2, o, fake, ctypes.byref(km), noise, ctypes.byref(opts), fake, wsb,
                                  None, None, fake, ctypes.byref(mu_p), ctypes.byref(ld_p), None)
    assert h.mvn_posterior(*args(None, 0.25, 1 << 30)) == -5
    assert h.mvn_posterior(*args(obs, 0.0, 1 << 30)) == -8
    assert h.mvn_posterior(*args(obs, 0.25, 16)) == -11
    wb = ctypes.c_size_t(0)
    assert h.mvn_posterior_workspace_bytes(10, 2, ctypes.byref(opts), ctypes.byref(wb)) == 0
    # m' = 64 (tile), bordered order 64 + 10 + 1 -> 128: the bordered matrix dominates
    assert wb.value >= 128 * 128 * 8
