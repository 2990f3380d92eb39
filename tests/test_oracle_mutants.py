"""The pins must be able to fail. Each case plants one plausible slip (a
dropped term, a wrong exponent, a wrong sign, a term at the wrong time
level) in a copy of the oracle's C source, builds the copy with gcc in a
temporary directory, and checks that the named pin rejects it. A site is
mutated at its first occurrence; the FP64 step precedes the FP32-gating step
in the file. The shipped oracle is never modified.
"""
import importlib.util
import os
import subprocess

import pytest

import test_oracle_pins as P

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE_DIR = os.path.join(os.path.dirname(HERE), "oracle")

# (name, original text, planted text, pin that must fail, its arguments)
MUTANTS = [
    ("leak reversal E_L -> E_K",
     "jion = (gna * P->ena + gk * P->ek) + P->gl * P->el;",
     "jion = (gna * P->ena + gk * P->ek) + P->gl * P->ek;",
     P.test_isolated_hh_compartment_rests_near_minus_65, {}),
    ("potassium n^4 -> n^3",
     "double gk = P->gkbar * (((nn * nn) * nn) * nn);",
     "double gk = P->gkbar * ((nn * nn) * nn);",
     P.test_driven_hh_compartment_converges_to_the_hh_ode, {}),
    ("sodium m^3 h -> m^2 h",
     "double gna = P->gnabar * (((m * m) * m) * h);",
     "double gna = P->gnabar * ((m * m) * h);",
     P.test_driven_hh_compartment_converges_to_the_hh_ode, {}),
    ("synaptic driving force sign",
     "r[i] = (o->af[b + i] * jion + gs[i] * P->e_syn) + iext;",
     "r[i] = (o->af[b + i] * jion - gs[i] * P->e_syn) + iext;",
     P.test_postsynaptic_potential_converges_to_the_conductance_ode,
     dict(e_syn=-80.0, precision=0)),
    ("synaptic conductance left off the diagonal",
     "gmem[i] = o->af[b + i] * gion + gs[i];",
     "gmem[i] = o->af[b + i] * gion;",
     P.test_postsynaptic_potential_converges_to_the_conductance_ode,
     dict(e_syn=0.0, precision=0)),
    ("injected current in every compartment",
     "double iext = (i == 0) ? o->iext[j] : 0.0;",
     "double iext = o->iext[j];",
     P.test_active_cable_converges_to_its_method_of_lines_ode, dict(precision=0)),
    ("no synaptic decay",
     "        o->g_d[k] = o->q * o->g_d[k];",
     "        o->g_d[k] = o->g_d[k];",
     P.test_single_event_conductance_is_w_q_power_k, {}),
    ("gates advanced at V^n instead of V^{n+1}",
     "        V[i] = r[i];\n        if (!o->mech[b + i]) continue;\n        orc_gates_update_d(V[i],",
     "        double vo = V[i];\n        V[i] = r[i];\n        if (!o->mech[b + i]) continue;\n"
     "        orc_gates_update_d(vo,",
     P.test_driven_hh_compartment_converges_to_the_hh_ode, {}),
    ("parent's diagonal takes the coupling twice",
     "        d[p[i]] -= o->e[b + i];",
     "        d[p[i]] -= 2.0 * o->e[b + i];",
     P.test_active_cable_converges_to_its_method_of_lines_ode, dict(precision=0)),
    ("parent's half-resistance replaced by the child's",
     "o->G[b + i] = 1.0 / (rhalf[b + i] + rhalf[b + parent[b + i]]);",
     "o->G[b + i] = 1.0 / (rhalf[b + i] + rhalf[b + i]);",
     P.test_diameter_step_converges_at_second_order, {}),
    ("implicit axial weight 1 instead of theta",
     "o->e[b + i] = -P->theta * o->G[b + i];",
     "o->e[b + i] = -o->G[b + i];",
     P.test_axial_time_stepping_order, dict(theta=0.5, order=2.0)),
    ("explicit axial weight 1 instead of 1 - theta",
     "    const double omt = 1.0 - P->theta;",
     "    const double omt = 1.0;",
     P.test_axial_time_stepping_order, dict(theta=0.5, order=2.0)),
    ("float path: leak reversal E_L -> E_K",
     "jion = (gna * ena + gk * ek) + gl * el;",
     "jion = (gna * ena + gk * ek) + gl * ek;",
     P.test_driven_hh_compartment_converges_to_the_hh_ode, {}),
    ("float path: synaptic conductance left off the diagonal",
     "gmem[i] = (double)(af * gion + gs[i]);",
     "gmem[i] = (double)(af * gion);",
     P.test_postsynaptic_potential_converges_to_the_conductance_ode,
     dict(e_syn=0.0, precision=1)),
    ("float path: synaptic driving force sign",
     "r[i] = (double)((af * jion + gs[i] * e_syn) + iext);",
     "r[i] = (double)((af * jion - gs[i] * e_syn) + iext);",
     P.test_postsynaptic_potential_converges_to_the_conductance_ode,
     dict(e_syn=-80.0, precision=1)),
    ("float path: injected current in every compartment",
     "float iext = (i == 0) ? (float)o->iext[j] : 0.0f;",
     "float iext = (float)o->iext[j];",
     P.test_active_cable_converges_to_its_method_of_lines_ode, dict(precision=1)),
    ("float path: gates advanced at V^n",
     "        V[i] = r[i];\n        if (!o->mech[b + i]) continue;\n        orc_gates_update_f((float)V[i],",
     "        double vo = V[i];\n        V[i] = r[i];\n        if (!o->mech[b + i]) continue;\n"
     "        orc_gates_update_f((float)vo,",
     P.test_driven_hh_compartment_converges_to_the_hh_ode, {}),
]


def load_oracle_from(lib_path, src_path):
    """A private instance of the oracle's Python wrapper bound to another
    build of the C source."""
    spec = importlib.util.spec_from_file_location("oracle_mutant_" + str(abs(hash(lib_path))),
                                                  os.path.join(ORACLE_DIR, "oracle.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod.SRC, mod.LIB, mod._lib = src_path, lib_path, None
    return mod


@pytest.mark.parametrize("name,orig,planted,pin,kwargs", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pin_rejects_planted_slip(tmp_path, name, orig, planted, pin, kwargs):
    src = open(os.path.join(ORACLE_DIR, "hines_oracle.c")).read()
    assert orig in src, "mutation site not found: " + name
    mutant_src = tmp_path / "mutant.c"
    mutant_src.write_text(src.replace(orig, planted, 1))   # the FP64 path comes first
    mutant_lib = tmp_path / "libmutant.so"
    from oracle import oracle as shipped
    subprocess.check_call(["gcc", *shipped.CFLAGS, str(mutant_src), "-o", str(mutant_lib), "-lm"])
    mod = load_oracle_from(str(mutant_lib), str(mutant_src))
    with pytest.raises(AssertionError):
        pin(mod, **kwargs)
