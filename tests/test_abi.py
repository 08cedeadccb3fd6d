"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/jk.h declares, and rejects bad input before touching
the device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2507_09772_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "jk.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(jk_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def jkmod():
    from paper_2507_09772_amd import jk
    jk.lib()
    return jk


def test_exports_every_declared_symbol(jkmod):
    names = _declared()
    assert "jk_build" in names and "jk_execute" in names
    for n in names:
        assert hasattr(jkmod.lib(), n), n


def _mol():
    return synth.workload("c0").mol


def _bad(**kw):
    m = _mol()
    d = dict(l=m.l.copy(), nprim=m.nprim.copy(), atom=m.atom.copy(), exps=m.exps.copy(), coefs=m.coefs.copy(),
             coords=m.coords.copy(), spherical=m.spherical)
    for k, v in kw.items():
        d[k] = v(d[k]) if callable(v) else v
    return synth.Molecule(**d)


def _set(arr, i, v):
    a = arr.copy()
    a[i] = v
    return a


@pytest.mark.parametrize("mol,code", [
    (lambda: _bad(l=lambda a: _set(a, 2, 9)), -1),
    (lambda: _bad(l=lambda a: _set(a, 2, 5)), -1),
    (lambda: _bad(nprim=lambda a: _set(a, 0, 0)), -1),
    (lambda: _bad(atom=lambda a: _set(a, 1, 99)), -1),
    (lambda: _bad(exps=lambda a: _set(a, 3, -1.0)), -1),
    (lambda: _bad(exps=lambda a: _set(a, 3, np.nan)), -1),
    (lambda: _bad(coefs=lambda a: _set(a, 0, np.inf)), -1),
    (lambda: _bad(coords=lambda a: _set(a, (0, 1), np.nan)), -1),
])
def test_plan_validation(jkmod, mol, code):
    with pytest.raises(jkmod.JKError) as e:
        jkmod.Plan(mol())
    assert e.value.code == code
    assert jkmod.lib().jk_last_error()


def test_bad_cutoff_and_null(jkmod):
    with pytest.raises(jkmod.JKError) as e:
        jkmod.Plan(_mol(), cutoff=-1.0)
    assert e.value.code == -1
    assert jkmod.lib().jk_plan_create(None, 1e-13, ctypes.byref(ctypes.c_void_p())) == -1
    assert jkmod.lib().jk_execute(None, None, 1, 3, 0, 0.0, 0.0, None, None, None) == -1
    assert jkmod.lib().jk_plan_info(None, None, None) == -1


def test_rys_eval_validation(jkmod):
    with pytest.raises(jkmod.JKError):
        jkmod.rys_eval(0, [1.0])
    with pytest.raises(jkmod.JKError):
        jkmod.rys_eval(3, [-1.0])
    with pytest.raises(jkmod.JKError):
        jkmod.rys_eval(10, [1.0])


def test_shipped_tuning_table_is_applied(jkmod):
    """Every entry of the shipped per-device table reaches the library (the
    table is read after the kernel classes have registered)."""
    path = os.path.join(ROOT, "paper_2507_09772_amd", "tune_gfx950.txt")
    rows = [list(map(int, l.split())) for l in open(path)
            if l.strip() and not l.startswith("#") and not l.startswith(("shape", "split"))]
    assert rows
    for r in rows:
        li, lj, lk, ll, pr, fam = r[:6]
        got, avail = jkmod.tune_get(li, lj, lk, ll, "fp32" if pr == 2 else "fp64")
        assert got == fam and avail & (1 << (fam - 1)), r
    # the task-shape lines parse and name canonical classes
    shapes = [l.split()[1:] for l in open(path) if l.startswith("shape")]
    for sh in shapes:
        assert len(sh) == 6
        jkmod.tune_set_shape(*map(int, sh))
    # the mixed-split lines likewise
    for sp in [l.split()[1:] for l in open(path) if l.startswith("split")]:
        assert len(sp) == 5 and sp[4] in ("0", "1")
        jkmod.tune_set_split(*map(int, sp))
    jkmod.tune_load(path)


def test_tuning_validation(jkmod):
    with pytest.raises(jkmod.JKError):
        jkmod.tune_set_split(0, 1, 0, 0, 0)   # not canonical
    with pytest.raises(jkmod.JKError):
        jkmod.tune_set_split(0, 0, 0, 0, 2)   # split is 0 or 1
    with pytest.raises(jkmod.JKError):
        jkmod.tune_set(0, 1, 0, 0, "fp64", 1)   # not canonical
    with pytest.raises(jkmod.JKError):
        jkmod.tune_set(0, 0, 0, 0, "fp64", 2)   # (ss|ss) has no family 2
    f, m = jkmod.tune_get(3, 3, 3, 3, "fp64")
    assert f == 2 and m == 2


def test_batch_validation(jkmod):
    L = jkmod.lib()
    h = ctypes.c_void_p()
    assert L.jk_batch_create(None, 1, 1, 0, 0.0, ctypes.byref(h)) == -1
    arr = (ctypes.c_void_p * 1)(None)
    assert L.jk_batch_create(arr, 0, 1, 0, 0.0, ctypes.byref(h)) == -1
    assert L.jk_batch_create(arr, 1, 0, 0, 0.0, ctypes.byref(h)) == -1
    assert L.jk_batch_create(arr, 1, 1, 7, 0.0, ctypes.byref(h)) == -1
    assert L.jk_batch_create(arr, 1, 1, 1, float("nan"), ctypes.byref(h)) == -1
    assert not h.value
    assert L.jk_batch_execute(None, None, None, None, None) == -1
    L.jk_batch_destroy(None)
