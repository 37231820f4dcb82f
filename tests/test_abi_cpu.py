"""The C-ABI library loads and exports every entry point include/rttda.h declares (no GPU needed),
and the host-side argument checks that run before any device work."""
import ctypes
import os
import re

import pytest

from paper_2601_16949_amd import rttda

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "rttda.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rttda_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = rttda.load()
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(rttda.EXPORTS), "binding and header disagree"


def test_version_and_variants():
    lib = rttda.load()
    assert lib.rttda_version().decode().startswith("rttda-gfx950")
    n = lib.rttda_exchange_variants(rttda.PREC_FP32)
    assert n >= 4
    names = [lib.rttda_exchange_variant_name(rttda.PREC_FP32, k).decode() for k in range(1, n + 1)]
    assert all(nm.startswith("f32") for nm in names) and len(set(names)) == len(names)
    assert lib.rttda_exchange_variant_name(rttda.PREC_FP32, n + 1).decode() == ""
    m = lib.rttda_exchange_variants(rttda.PREC_MIXED_BF16)
    mixed = [lib.rttda_exchange_variant_name(rttda.PREC_MIXED_BF16, k).decode() for k in range(1, m + 1)]
    assert m >= 4 and all(nm.startswith("bf16") for nm in mixed) and len(set(mixed)) == m
    assert lib.rttda_exchange_variants(7) == 0


def desc(o=10, v=40, nq=120, prec=rttda.PREC_FP32, bd=rttda.F32, max_rhs=3):
    d = rttda.CDesc()
    d.n_occ, d.n_virt, d.n_aux = o, v, nq
    d.precision, d.b_dtype, d.max_rhs = prec, bd, max_rhs
    d.cx = 0.2
    return d


def ws_bytes(d):
    n = ctypes.c_size_t(0)
    st = rttda.load().rttda_workspace_bytes(ctypes.byref(d), ctypes.byref(n))
    return st, n.value


def test_workspace_query_and_validation():
    st, n = ws_bytes(desc())
    assert st == rttda.OK and n > 0
    st2, n2 = ws_bytes(desc(max_rhs=6))
    assert st2 == rttda.OK and n2 > n  # grows with the RHS count
    for bad in (desc(o=0), desc(v=0), desc(nq=-1), desc(max_rhs=0), desc(max_rhs=5000),
                desc(prec=rttda.PREC_FP32, bd=rttda.BF16), desc(prec=rttda.PREC_MIXED_BF16, bd=rttda.F32),
                desc(prec=9)):
        st, _ = ws_bytes(bad)
        assert st == rttda.E_INVAL
        assert rttda.load().rttda_last_error().decode() != ""


def test_create_rejects_null_pointers_before_any_device_work():
    d = desc()
    h = ctypes.c_void_p()
    st = rttda.load().rttda_create(ctypes.byref(d), ctypes.byref(h))
    assert st == rttda.E_INVAL
    assert "NULL" in rttda.load().rttda_last_error().decode()
    assert rttda.load().rttda_destroy(None) == rttda.E_INVAL


def test_packaged_autotune_choices_name_variants_of_this_build():
    """Every packaged autotune entry (key p<precision>_o.._v.._nq.._r<nrhs>) names an exchange
    variant the library has for that precision, with a positive split count."""
    from paper_2601_16949_amd import autotune

    lib = rttda.load()
    cache = autotune.load_cache()
    assert cache
    for key, e in cache.items():
        prec = int(key.split("_")[0][1:])
        names = [lib.rttda_exchange_variant_name(prec, k).decode()
                 for k in range(1, lib.rttda_exchange_variants(prec) + 1)]
        assert e["name"] in names, (key, e["name"])
        assert int(e["splits"]) >= 1


def test_autotune_keys_carry_the_integrator():
    """RK4 and the split operator launch the exchange on 2R and R slices, so their tuned choices
    are kept apart; the packaged split-operator entries name the same shapes as RK4 ones."""
    from types import SimpleNamespace

    from paper_2601_16949_amd import autotune

    ctx = SimpleNamespace(desc=SimpleNamespace(precision=1, n_occ=60, n_virt=400, n_aux=1500))
    assert autotune._key(ctx, 3) == "p1_o60_v400_nq1500_r3"
    assert autotune._key(ctx, 3, "sso") == "p1_o60_v400_nq1500_r3_sso"
    cache = autotune.load_cache()
    for key in cache:
        if key.endswith("_sso"):
            assert key[: -len("_sso")] in cache, key


def test_serving_stream_and_footprint_host_logic():
    """The serving workload stream (o ~ U{10..48} here, v = floor(7.5 o), N_Q = 20 o, Poisson
    arrivals) and the footprint used for admission: increasing arrival times, the stated size
    rules, and a footprint that covers the factors, the library's own workspace and the state."""
    import math

    import numpy as np

    from paper_2601_16949_amd import inputs as I
    from paper_2601_16949_amd import serve

    reqs = I.serving_requests(400, rate=20.0, o_min=10, o_max=48)
    t = np.array([r.arrival for r in reqs])
    assert np.all(np.diff(t) > 0)
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert abs(gaps.mean() - 1 / 20.0) < 0.2 / 20.0  # exponential gaps of mean 1/rate
    for r in reqs:
        o = r.shape.o
        assert 10 <= o <= 48 and r.shape.v == math.floor(7.5 * o) and r.shape.nq == 20 * o
        assert 500 <= r.n_steps <= 8000 and r.shape.storage == "bf16"
        assert r.pulse.kind in (I.PULSE_DELTA, I.PULSE_GAUSS)
    kinds = [r.pulse.kind for r in reqs]
    assert 0.4 < kinds.count(I.PULSE_DELTA) / len(kinds) < 0.6
    sh = reqs[0].shape
    fp = serve.footprint(sh, 1000, "mixed")
    ws = rttda.workspace_bytes(sh.o, sh.v, sh.nq, "mixed", 1)
    factors = sh.nq * (sh.o * sh.v + sh.o ** 2 + sh.v ** 2) * 2
    assert fp >= ws + factors + 2 * sh.o * sh.v * 8 + 1001 * 8
    assert serve.footprint(sh, 2000, "mixed") - fp == 1000 * 8


def test_pool_host_logic_without_device_work():
    """The serving pool's bookkeeping needs no device: an empty pool reports zero use, steps
    nothing, refuses unknown slots and NULL arguments with RTTDA_E_INVAL, and is destroyed."""
    lib = rttda.load()
    h = ctypes.c_void_p()
    assert lib.rttda_pool_create(1 << 30, ctypes.byref(h)) == rttda.OK
    used, active = ctypes.c_size_t(7), ctypes.c_int32(7)
    assert lib.rttda_pool_usage(h, ctypes.byref(used), ctypes.byref(active)) == rttda.OK
    assert used.value == 0 and active.value == 0
    issued = ctypes.c_int32(-1)
    assert lib.rttda_pool_step(h, 10, ctypes.byref(issued)) == rttda.OK and issued.value == 0
    assert lib.rttda_pool_step(h, 0, None) == rttda.E_INVAL
    done, fin = ctypes.c_int64(), ctypes.c_int32()
    assert lib.rttda_pool_poll(h, 0, ctypes.byref(done), ctypes.byref(fin)) == rttda.E_INVAL
    assert lib.rttda_pool_release(h, 3) == rttda.E_INVAL
    slot = ctypes.c_int32()
    assert lib.rttda_pool_admit(h, None, 1, None, 0.05, 10, rttda.INTEG_RK4, None, None, None, 0,
                                ctypes.byref(slot)) == rttda.E_INVAL
    assert lib.rttda_pool_create(1, None) == rttda.E_INVAL
    assert lib.rttda_pool_destroy(h) == rttda.OK
    assert lib.rttda_pool_destroy(None) == rttda.E_INVAL


def test_sigma_noalloc_host_checks():
    """rttda_sigma_noalloc refuses bad arguments and shapes beyond its static scratch before any
    device work (the pointers below are never dereferenced)."""
    lib = rttda.load()
    f = (ctypes.c_double * 3)(0.0, 0.0, 0.0)
    dirs = (ctypes.c_double * 9)(0, 0, 1, 0, 0, 1, 0, 0, 1)
    fake = 1 << 20
    assert lib.rttda_sigma_noalloc(None, 1, f, dirs, fake, fake, fake, fake) == rttda.E_INVAL
    d = desc(o=240, v=1800, nq=8, max_rhs=3)
    d.e_occ = d.e_virt = d.mu = d.b_ov = d.b_oo = d.b_vv = fake
    assert lib.rttda_sigma_noalloc(ctypes.byref(d), 3, f, dirs, fake, fake, fake, fake) == rttda.E_NOMEM
    assert "static scratch" in lib.rttda_last_error().decode()
    assert lib.rttda_sigma_noalloc(ctypes.byref(d), 65, f, dirs, fake, fake, fake, fake) == rttda.E_INVAL
    assert lib.rttda_sigma_noalloc(ctypes.byref(d), 1, f, dirs, fake + 8, fake, fake, fake) == rttda.E_INVAL
