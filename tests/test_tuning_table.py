"""The MI355X tuning table shipped with the package (the library autotuner's cache format) and the
way bench.py starts from it.  Host only."""

import argparse
import importlib.util
import os

import pytest

from paper_2201_01257_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TABLE = os.path.join(ROOT, "paper_2201_01257_amd", "tuning", "mi355x.txt")

lib = _lib.load()


def _count(precision):
    n = 0
    while lib.tamm_config_name(precision, n):
        n += 1
    return n


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_table_lines_are_well_formed():
    n_f64 = _count(0)
    n_max = max(_count(p) for p in range(4))
    assert n_f64 >= 10
    lines = [l.split() for l in open(TABLE) if l.strip()]
    assert lines
    sigs = set()
    for sig, kind, config, k_splits, grid, ms in lines:
        assert len(sig) == 16 and int(sig, 16) >= 0
        assert (sig, kind) not in sigs  # one entry per plan or group class
        sigs.add((sig, kind))
        config, k_splits, grid, ms = int(config), int(k_splits), int(grid), float(ms)
        if kind == "plan2":  # configuration, K splits, die chunk + tile order * 2^24
            assert 0 <= config < n_max
            assert k_splits in (1, 2, 4, 8)
            assert grid & 0xFFFFFF in (0, 16, 32, 64, 128) and grid >> 24 in (0, 1)
            assert 0.0 < ms < 1e4
        else:  # a group's layout class: configuration (-1: empty class) and persistent grid
            assert kind.startswith("group") and 0 <= int(kind[5:]) < 8
            assert -1 <= config < n_f64 and grid >= 0 and k_splits == 1
            assert ms > 0.0


def test_bench_starts_from_a_private_copy(tmp_path):
    bench = _bench()
    args = argparse.Namespace(tune_cache=None)
    src = bench.resolve_tune_cache(args)
    try:
        assert src.startswith("tuning table") and args.tune_cache != TABLE
        assert open(args.tune_cache).read() == open(TABLE).read()
    finally:
        os.unlink(args.tune_cache)
    args = argparse.Namespace(tune_cache="none")
    assert bench.resolve_tune_cache(args) == "autotuned in the run" and args.tune_cache == ""
    own = str(tmp_path / "cache.txt")
    args = argparse.Namespace(tune_cache=own)
    assert bench.resolve_tune_cache(args) == "cache file " + own and args.tune_cache == own
