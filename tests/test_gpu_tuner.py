"""The tile configuration of the FP64 chi0 contraction changes speed, never results.

Every configuration (64-wide tiles with 8, 16, 32 rows of B per LDS step; 128-wide tiles
with 16; 64-wide tiles with 16-row steps contracting two frequencies of a q per
workgroup) runs the same sequence of 4-row MFMA steps in the same row order on the same
weighted products, so with one row split chi0 is bit-for-bit the same for all; each must
match the oracle to 1e-12 (Frobenius, relative).  The paired configuration is checked
through whole energies (the only calls with several points per launch), with odd
frequency counts so that pairs are left single at the end of every q.  The tuner must
record one choice per shape bucket, persist it when asked, and leave E within 1e-12 of a
run at the fixed default configuration.
"""
import os
import sys

import numpy as np
import pytest

from oracle import rpa_oracle as orc
from paper_2505_06021_amd import inputs

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-test] {msg}", file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    from paper_2505_06021_amd import rpa
    c = rpa.Context(0)
    yield c
    c.close()


def tall_system():
    # M = 4 * 8 * 150 = 4800 rows (more than the 4096 rows the tuner times), N = 150
    return inputs.make_system("tall", (2, 2, 1), 8, 150, 150, 3, 41, is_complex=True)


CFGS = ("t64k8", "t64k16", "t64k32", "t128k16", "t64k16w2")


@pytest.mark.parametrize("naux", [150, 257])
def test_chi0_every_configuration_identical_and_exact(ctx, monkeypatch, naux):
    # N = 150 and 257: ragged 64- and 128-wide tiles (257 leaves a one-column tile)
    s = inputs.make_system("tall", (2, 2, 1), 8, 150, naux, 3, 41, is_complex=True)
    ref = orc.chi0(s, 1, s.omega[1])
    monkeypatch.setenv("RPA_CHI0_KSPLIT", "1")   # the configurations' own split counts differ
    got = {}
    for cfg in CFGS:
        say(f"chi0 configuration {cfg} N={naux}")
        monkeypatch.setenv("RPA_CHI0_CFG", cfg)
        got[cfg] = ctx.chi0(s, 1, s.omega[1])
        err = np.linalg.norm(got[cfg] - ref) / np.linalg.norm(ref)
        assert err <= 1e-12, (cfg, err)
    for cfg in CFGS[1:]:
        assert np.array_equal(got[cfg], got[CFGS[0]]), cfg


def test_energy_every_configuration_matches_oracle(ctx, monkeypatch):
    s = inputs.make_system("cfgE", (2, 2, 1), 3, 7, 150, 4, 32, is_complex=True, sigma=0.15)
    E_ref = orc.energy(s)[0]
    for cfg in CFGS:
        say(f"energy configuration {cfg}")
        monkeypatch.setenv("RPA_CHI0_CFG", cfg)
        E, _ = ctx.energy(s)
        assert abs(E - E_ref) <= 1e-10 * abs(E_ref), cfg


def test_legacy_depth_variable(ctx, monkeypatch):
    s = tall_system()
    monkeypatch.setenv("RPA_CHI0_CFG", "t64k32")
    a = ctx.chi0(s, 0, s.omega[0])
    monkeypatch.delenv("RPA_CHI0_CFG")
    monkeypatch.setenv("RPA_CHI0_KT", "32")
    b = ctx.chi0(s, 0, s.omega[0])
    assert np.array_equal(a, b)


def test_tuner_records_and_persists_choice(ctx, monkeypatch, tmp_path):
    from paper_2505_06021_amd import rpa
    s = inputs.make_system("tune", (2, 2, 1), 3, 7, 150, 5, 31, is_complex=True, sigma=0.15)
    monkeypatch.setenv("RPA_CHI0_CFG", "t64k16")
    say("energy at the fixed default configuration")
    e_fixed, eps_fixed = ctx.energy(s)
    monkeypatch.delenv("RPA_CHI0_CFG")
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("RPA_TUNE_CACHE", str(cache))
    say("energy with the tuner")
    e_tuned, eps_tuned = ctx.energy(s)
    choices = {k: v for k, v in rpa.tuned().items() if k.startswith("f64_")}
    assert choices, "the tuner recorded no choice"
    assert all(v in CFGS for v in choices.values())
    assert any(k.startswith("f64_c_N192_") for k in choices), choices
    assert abs(e_tuned - e_fixed) <= 1e-12 * abs(e_fixed)
    assert np.max(np.abs(eps_tuned - eps_fixed)) <= 1e-12 * np.max(np.abs(eps_fixed))
    e_ref = orc.energy(s)[0]
    assert abs(e_tuned - e_ref) <= 1e-10 * abs(e_ref)
    if cache.exists():   # written when the bucket was tuned in this test's lifetime
        lines = dict(l.split() for l in cache.read_text().splitlines())
        assert all(v in CFGS for k, v in lines.items() if k.startswith("f64_"))


def test_fp32_tile_tuner_records_choice(ctx, monkeypatch):
    from paper_2505_06021_amd import rpa
    monkeypatch.delenv("RPA_F32_TILE", raising=False)
    s = inputs.make_system("tune32", (2, 2, 1), 3, 7, 150, 4, 33, is_complex=True, sigma=0.15)
    say("energy fp32 with the tile tuner")
    E, _ = ctx.energy(s, prec=1)
    choices = {k: v for k, v in rpa.tuned().items() if k.startswith("f32_")}
    assert choices and all(v in ("t64", "t128", "t64w2") for v in choices.values()), choices
    assert abs(E - orc.energy(s)[0]) <= 1e-6


@pytest.mark.parametrize("nw,is_complex", [(3, True), (5, True), (4, False)])
def test_paired_frequencies_match_single_point_kernel(ctx, monkeypatch, nw, is_complex):
    # several q with an odd (or even) number of frequencies each: the pair table of a
    # batch pairs the frequencies of one q and leaves the last one of an odd q single;
    # these systems are too short for a row split, so the per-point energies equal the
    # single-point kernel's bit for bit
    s = inputs.make_system("pair", (2, 2, 1), 3, 9, 150, nw, 37, is_complex=is_complex, sigma=0.15)
    monkeypatch.setenv("RPA_CHI0_CFG", "t64k16")
    say(f"energy nw={nw} complex={is_complex}: single-point kernel")
    e1, g1 = ctx.energy(s)
    monkeypatch.setenv("RPA_CHI0_CFG", "t64k16w2")
    say("  paired kernel")
    e2, g2 = ctx.energy(s)
    e_ref, g_ref = orc.energy(s)
    assert abs(e2 - e_ref) <= 1e-10 * abs(e_ref)
    for q in range(s.nq):
        assert np.max(np.abs(g2[q] - g_ref[q])) <= 1e-10 * np.max(np.abs(g_ref[q]))
    assert np.array_equal(g2, g1)


@pytest.mark.parametrize("cfg", ["t64k16", "t64k16w2", "t128k16"])
def test_row_splits_agree(ctx, monkeypatch, cfg):
    # one to four row splits of every contraction launch (the later splits' sums land in
    # partial planes added in split order): each equals the oracle, and the per-point
    # energies of different split counts differ only by the reordered FP64 sums
    s = inputs.make_system("splits", (2, 2, 1), 8, 150, 200, 3, 43, is_complex=True, sigma=0.15)
    e_ref, g_ref = orc.energy(s)
    monkeypatch.setenv("RPA_CHI0_CFG", cfg)
    base = None
    for ks in (1, 2, 3, 4):
        monkeypatch.setenv("RPA_CHI0_KSPLIT", str(ks))
        say(f"energy {cfg} with {ks} row splits")
        e, g = ctx.energy(s)
        assert abs(e - e_ref) <= 1e-10 * abs(e_ref), (ks, e, e_ref)
        for q in range(s.nq):
            assert np.max(np.abs(g[q] - g_ref[q])) <= 1e-10 * np.max(np.abs(g_ref[q])), (ks, q)
        if base is None:
            base = g
        else:
            assert np.max(np.abs(g - base)) <= 1e-12 * np.max(np.abs(base)), ks


@pytest.mark.parametrize("prec", [0, 1])
def test_paired_kernels_on_device_inputs(ctx, monkeypatch, prec):
    # B and V^(1/2) resident on the device (the contraction reads the caller's slab of
    # each q directly): the paired FP64 and FP32 kernels give the single-point kernels'
    # energies bit for bit
    s = inputs.make_system("pairdev", (2, 2, 1), 3, 9, 150, 5, 53, is_complex=True, sigma=0.15)
    var, single, paired = ("RPA_CHI0_CFG", "t64k16", "t64k16w2") if prec == 0 else ("RPA_F32_TILE", "64", "64w2")
    monkeypatch.setenv(var, single)
    say(f"device inputs prec={prec}: single-point kernel")
    e1, g1 = ctx.energy(s, prec=prec, device=True)
    monkeypatch.setenv(var, paired)
    say("  paired kernel")
    e2, g2 = ctx.energy(s, prec=prec, device=True)
    assert np.array_equal(g1, g2)
    assert abs(e2 - orc.energy(s)[0]) <= (1e-10 * abs(e2) if prec == 0 else 1e-6)


@pytest.mark.parametrize("is_complex", [True, False])
@pytest.mark.parametrize("naux", [40, 64, 65, 129])
@pytest.mark.parametrize("prec", [0, 1])
def test_paired_kernels_small_and_ragged_tile_grids(ctx, monkeypatch, naux, prec, is_complex):
    # one tile (N <= 64: no off-diagonal tile at all), a ragged second tile row, and a
    # one-column third tile row: the paired kernels' workgroup order (off-diagonal tiles
    # first, diagonal tiles last) must cover every tile of every pair once
    s = inputs.make_system("pairgrid", (2, 2, 1), 3, 7, naux, 3, 59, is_complex=is_complex, sigma=0.15)
    var, single, paired = ("RPA_CHI0_CFG", "t64k16", "t64k16w2") if prec == 0 else ("RPA_F32_TILE", "64", "64w2")
    monkeypatch.setenv(var, single)
    say(f"N_aux {naux} prec={prec}: single-point kernel")
    e1, g1 = ctx.energy(s, prec=prec)
    monkeypatch.setenv(var, paired)
    say("  paired kernel")
    e2, g2 = ctx.energy(s, prec=prec)
    assert np.array_equal(g1, g2)
    e_ref = orc.energy(s)[0]
    assert abs(e2 - e_ref) <= (1e-10 * abs(e_ref) if prec == 0 else 1e-6)


@pytest.mark.parametrize("prec", [0, 1])
def test_single_point_chi0_row_splits(ctx, monkeypatch, prec):
    # rpa_chi0 splits the rows of its one point so that the launch fills the GPU (up to
    # 16 splits of at least 512 rows; the later splits' sums go to partial planes added
    # in split order): every split count agrees with the oracle and with one split
    s = inputs.make_system("chi0split", (2, 2, 1), 8, 150, 200, 3, 61, is_complex=True)   # M = 4800
    ref = orc.chi0(s, 1, s.omega[1])
    tol = 1e-12 if prec == 0 else 1e-6
    monkeypatch.setenv("RPA_CHI0_KSPLIT", "1")
    one = ctx.chi0(s, 1, s.omega[1], prec=prec)
    for ks in ("2", "5", "9", "16"):
        monkeypatch.setenv("RPA_CHI0_KSPLIT", ks)
        say(f"chi0 prec={prec} with {ks} row splits")
        got = ctx.chi0(s, 1, s.omega[1], prec=prec)
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= tol, ks
        assert np.linalg.norm(got - one) / np.linalg.norm(one) <= (1e-14 if prec == 0 else 1e-6), ks
        assert np.abs(got - got.conj().T).max() == 0.0
    monkeypatch.delenv("RPA_CHI0_KSPLIT")
    say("  the launch's own split count")
    got = ctx.chi0(s, 1, s.omega[1], prec=prec)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= tol
