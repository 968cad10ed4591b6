"""Front end for the stencil description language (Sec. 3.2): DSL programs
written for the four models parse into exactly the built-in model stencils
and the oracle's model terms, constants and per-site coefficients map to the
on-site block and field modes, and malformed programs are rejected with the
offending line."""

import os

import numpy as np
import pytest

import paper_1708_09689_amd as pv
from oracle import models

HERE = os.path.join(os.path.dirname(__file__), "golden", "dsl")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(pv.LIB_PATH):
        pytest.skip("libpvdtm.so not built")
    return pv.lib()


def read(name):
    return open(os.path.join(HERE, name)).read()


def by_offset(st):
    return {tuple(int(v) for v in o): B for o, B in zip(st["offsets"], st["blocks"])}


def oracle_descriptor(model):
    out = {}
    for e, A in model.hops:
        out[tuple(-np.asarray(e))] = A
        out[tuple(np.asarray(e))] = A.conj().T
    return out


@pytest.mark.parametrize("name,code,params,model,pot,field", [
    ("ti.dsl", pv.PV_MODEL_TI, [1.0, 2.0, 0, 0], models.topological_insulator(1.0, 2.0), pv.PV_POT_SITE, 1),
    ("graphene2.dsl", pv.PV_MODEL_GRAPHENE2, [1.0], models.graphene_two_site(1.0), pv.PV_POT_SITE, 1),
    ("graphene4.dsl", pv.PV_MODEL_GRAPHENE4, [1.0], models.graphene_four_site(1.0), pv.PV_POT_ORBITAL, 1),
    ("weyl.dsl", pv.PV_MODEL_WEYL, [np.pi / 2], models.weyl_semimetal(), pv.PV_POT_SITE, 2),
])
def test_programs_equal_model_stencils(lib, name, code, params, model, pot, field):
    st = pv.pv_dsl_stencil(read(name))
    ref = pv.pv_model_stencil(code, params)
    assert st["n_orb"] == ref["n_orb"] and st["dim"] == ref["dim"]
    assert st["pot_mode"] == pot and st["field"] == field
    a, b = by_offset(st), by_offset(ref)
    assert set(a) == set(b)
    for off in a:
        assert np.array_equal(a[off], b[off]), off
    assert np.array_equal(st["onsite"], ref["onsite"])
    orc = oracle_descriptor(model)
    for off in a:
        assert np.abs(a[off] - orc[off]).max() < 1e-15
    assert np.abs(st["onsite"] - model.onsite).max() < 1e-15


def test_parsed_stencil_selects_the_compiled_family(lib):
    for name, fam in [("ti.dsl", 1), ("graphene2.dsl", 2), ("graphene4.dsl", 3), ("weyl.dsl", 4)]:
        st = pv.pv_dsl_stencil(read(name))
        L = (4, 4, 4) if st["dim"] == 3 else (4, 4)
        assert pv.Lattice(L, (1, 1, 1), st).family == fam


def test_constant_coefficients_from_caller(lib):
    st = pv.pv_dsl_stencil(read("ti.dsl"), coeff_const=[1.5])      # m = 1.5 instead of the default 2
    ref = pv.pv_model_stencil(pv.PV_MODEL_TI, [1.0, 1.5, 0, 0])
    assert np.allclose(np.diag(st["onsite"])[:2], [1.5, 1.5]) and np.allclose(np.diag(st["onsite"])[2:], [-2, -2])
    assert np.array_equal(by_offset(st)[(1, 0, 0)], by_offset(ref)[(1, 0, 0)])


def test_complex_values_and_layout_freedom(lib):
    text = """
# comments, blank lines, no row labels, trailing separators
dim 2
size 2

nn 1 0
1|1.5-2e-1i;
0|-3i;  1|+0.25i ;
nn -1 0
l0; 1|-3i
l1; 0|1.5+0.2i; 1|-0.25i
nn 0 0
l0; 0|1
l1;
"""
    st = pv.pv_dsl_stencil(text)
    B = by_offset(st)
    assert B[(1, 0, 0)][0, 1] == 1.5 - 0.2j and B[(1, 0, 0)][1, 0] == -3j and B[(1, 0, 0)][1, 1] == 0.25j
    assert st["pot_mode"] == pv.PV_POT_NONE and st["field"] == 0
    assert st["onsite"][0, 0] == 1 and st["onsite"][1, 1] == 0


@pytest.mark.parametrize("text,where", [
    ("dim 2\nsize 2\nfoo 3\n", "line 3"),
    ("nn 1 0\n", "line 1"),
    ("dim 2\nsize 2\nnn 1 0\nl0; 1|1\n", "line 3"),                   # block ends early
    ("dim 2\nsize 2\nnn 1 0\nl0; 2|1\nl1;\n", "line 4"),              # column out of range
    ("dim 2\nsize 2\nnn 1 0\nl1; 1|1\nl0;\n", "line 4"),              # wrong row label
    ("dim 2\nsize 2\nnn 2 0\nl0;\nl1;\n", "line 3"),                  # offset outside {-1, 0, 1}
    ("dim 3\nsize 2\nnn 1 0\nl0;\nl1;\n", "line 3"),                  # dim 3 needs three offsets
    ("dim 2\nsize 2\nnn 1 0\nl0;\nl1;\nnn 1 0\nl0;\nl1;\n", "line 6"),  # offset twice
    ("dim 2\nsize 2\nn_coeff_variable 1\nnn 1 0\nl0; 0|v|0\nl1;\n", "line 5"),  # v off the on-site block
    ("dim 2\nsize 2\nn_coeff_const 1\nnn 0 0\nl0; 0|c|0\nl1;\n", "line 5"),    # constant without a value
    ("dim 2\nsize 2\nnn 0 0\nl0; 0|x|1\nl1;\n", "line 4"),            # unknown type
    ("dim 2\nsize 2\nnn 0 0\nl0; 0|1; 0|2\nl1;\n", "line 4"),         # entry twice
    ("dim 2\nsize 2\nnn 0 0\nl0; 0|1z\nl1;\n", "line 4"),             # bad value
])
def test_malformed_programs(lib, text, where):
    with pytest.raises(pv.PvError) as e:
        pv.pv_dsl_stencil(text)
    assert e.value.status == 1
    assert where in str(e.value)


def test_unsupported_field_shapes(lib):
    half = "dim 2\nsize 2\nn_coeff_variable 1\nnn 0 0\nl0; 0|v|0\nl1;\n"          # not every orbital
    mixed = "dim 2\nsize 2\nn_coeff_variable 1\nn_coeff_rand 1\nnn 0 0\nl0; 0|v|0\nl1; 1|r|0\n"
    perm = "dim 2\nsize 2\nn_coeff_variable 2\nnn 0 0\nl0; 0|v|1\nl1; 1|v|0\n"
    for t in (half, mixed, perm):
        with pytest.raises(pv.PvError) as e:
            pv.pv_dsl_stencil(t)
        assert e.value.status == 2
