"""The tile configuration of the FP64 chi0 contraction changes speed, never results.

Every configuration (64-wide tiles with 8, 16, 32 rows of B per LDS step; 128-wide tiles
with 16) runs the same sequence of 4-row MFMA steps in the same row order, so with one
row split chi0 is bit-for-bit the same for all; each must match the oracle to 1e-12
(Frobenius, relative).  The tuner must record one choice per shape bucket, persist it
when asked, and leave E within 1e-12 of a run at the fixed default configuration.
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


CFGS = ("t64k8", "t64k16", "t64k32", "t128k16")


@pytest.mark.parametrize("naux", [150, 257])
def test_chi0_every_configuration_identical_and_exact(ctx, monkeypatch, naux):
    # N = 150 and 257: ragged 64- and 128-wide tiles (257 leaves a one-column tile)
    s = inputs.make_system("tall", (2, 2, 1), 8, 150, naux, 3, 41, is_complex=True)
    ref = orc.chi0(s, 1, s.omega[1])
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
    assert choices and all(v in ("t64", "t128") for v in choices.values()), choices
    assert abs(E - orc.energy(s)[0]) <= 1e-6
