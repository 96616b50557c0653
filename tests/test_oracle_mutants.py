"""The oracle's pins catch plausible mistakes in the oracle.

Each case plants one mistake in a copy of the oracle (a dropped term, a wrong
sign, an operand swapped, an off-by-one range, the wrong R or the wrong tie
rule), on the CPU: C mistakes in a mutated copy of oracle/orc.c compiled to a
temporary library, Python ones in a mutated copy of the function.  The pin
tests of tests/test_oracle_pins.py then run against the mutant, and at least
one must fail.  The unmutated oracle passes all of them (that file's own run).
"""
import inspect
import itertools
import os
import subprocess
import sys

import pytest

import oracle as orc

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import test_oracle_pins as pins  # noqa: E402

# (name, original text, planted text): each original occurs exactly once in orc.c
C_MUTANTS = [
    ("plantard result not negated",
     "*out = p->variant == ORC_CLASSIC ? c : (c == 0 ? 0 : N - c);",
     "*out = c;"),
    ("Plantard reduces modulo 2^w instead of 2^(2w)",
     "        logR = 2 * w;\n        break;\n    }\n    case ORC_SIGNED_PLANTARD:",
     "        logR = w;\n        break;\n    }\n    case ORC_SIGNED_PLANTARD:"),
    ("R instead of R^{-1}",
     "p->rinv = orc_inv_mod(pow2_mod(logR, N), N);",
     "p->rinv = pow2_mod(logR, N);"),
    ("signed Montgomery tie on the wrong side of R/2",
     "(a0 < ((i128)1 << (w - 1)))",
     "(a0 <= ((i128)1 << (w - 1)))"),
    ("signed Montgomery window independent of a0",
     "(i128)((N + 1) / 2);",
     "(i128)((N - 1) / 2);"),
    ("high word by truncating division instead of floor",
     "i128 a1 = T >> w; /* arithmetic shift = floor division */",
     "i128 a1 = T / ((i128)1 << w);"),
    ("least absolute remainder off by one",
     "return x <= (N - 1) / 2 ? (int64_t)x : (int64_t)((i128)x - (i128)N);",
     "return x < (N - 1) / 2 ? (int64_t)x : (int64_t)((i128)x - (i128)N);"),
    ("negative remainders left negative",
     "    if (r < 0)\n        r += (i128)N;\n    return (uint64_t)r;",
     "    return (uint64_t)r;"),
    ("classic input bound R N taken as R",
     "u128 RN = (u128)N << p->w;",
     "u128 RN = (u128)1 << p->w;"),
    ("exponentiation multiplies by the base instead of its square",
     "acc = (acc * b) % N;",
     "acc = (acc * base) % N;"),
    ("exponentiation with 0^0 = 0",
     "u128 acc = 1;",
     "u128 acc = base ? 1 : 0;"),
    ("inverse transform without the 1/n factor",
     "ninv = orc_inv_mod(n % N, N);",
     "ninv = 1;"),
    ("transform exponent j + k instead of j k",
     "powers[(j * k) & (n - 1)]",
     "powers[(j + k) & (n - 1)]"),
    ("inverse transform with w instead of w^{-1}",
     "        wi = orc_inv_mod(wi, N);\n        if (!wi)",
     "        if (!wi)"),
]

# (name, function, original text, planted text) for the oracle's Python functions
PY_MUTANTS = [
    ("CRT coefficient without the inverse of M_j", "crt",
     "coef.append(Mj * _egcd_inverse(Mj % N, N))", "coef.append(Mj)"),
    ("CRT result not reduced modulo M", "crt",
     "for j in range(k)) % M for i in range(n)]", "for j in range(k)) for i in range(n)]"),
    ("least absolute remainder tie taken upward", "mods",
     "return r - n if 2 * r >= n else r", "return r - n if 2 * r > n else r"),
    ("N' as N^{-1} instead of R - N^{-1}", "constants",
     '"nprime": R - ninv,', '"nprime": ninv,'),
    ("Algorithm 4 offset 2^alpha taken as 2^(alpha - 1)", "sigpredc2_steps",
     "q = (m >> n) + (1 << alpha)", "q = (m >> n) + (1 << (alpha - 1))"),
]


def _param_sets(fn):
    """The keyword sets pytest would call a pin test with (no fixtures)."""
    sig = inspect.signature(fn)
    marks = [m for m in getattr(fn, "pytestmark", []) if m.name == "parametrize"]
    axes = []
    for m in marks:
        names = [s.strip() for s in m.args[0].split(",")] if isinstance(m.args[0], str) else list(m.args[0])
        vals = [v if len(names) > 1 else (v,) for v in m.args[1]]
        vals = [tuple(getattr(v, "values", v)) for v in vals]
        axes.append([dict(zip(names, v)) for v in vals])
    if set(sig.parameters) - {k for ax in axes for d in ax for k in d}:
        return []  # needs a fixture: not run here
    return [{k: v for d in combo for k, v in d.items()} for combo in itertools.product(*axes)] or [{}]


def _first_failing_pin():
    """Runs the pins in file order, the exhaustive one (seconds) last; the name of
    the first one that fails, or None."""
    tests = [(n, f) for n, f in vars(pins).items() if n.startswith("test_") and inspect.isfunction(f)]
    tests.sort(key=lambda t: "exhaustive" in t[0])
    for name, fn in tests:
        for kw in _param_sets(fn):
            try:
                fn(**kw)
            except Exception:  # an assertion, or the mutant refusing valid input
                return name
    return None


def _compile_mutant(tmp_path, original, planted):
    src = open(orc._SRC).read()
    assert src.count(original) == 1, "mutation site not unique: %r" % original
    path = tmp_path / "orc_mutant.c"
    path.write_text(src.replace(original, planted))
    lib = tmp_path / "liborc_mutant.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-w", "-shared", "-fPIC", "-o", str(lib), str(path)], check=True)
    return str(path), str(lib)


@pytest.mark.parametrize("name,original,planted", C_MUTANTS, ids=[m[0] for m in C_MUTANTS])
def test_c_mutant_is_caught(name, original, planted, tmp_path, monkeypatch):
    src, lib = _compile_mutant(tmp_path, original, planted)
    monkeypatch.setattr(orc, "_SRC", src)
    monkeypatch.setattr(orc, "_LIB", lib)
    monkeypatch.setattr(orc, "_lib", None)
    caught = _first_failing_pin()
    assert caught is not None, "no pin catches: " + name


def _mutated_function(fname, original, planted):
    src = inspect.getsource(getattr(orc, fname))
    assert src.count(original) == 1, "mutation site not unique: %r" % original
    ns = dict(vars(orc))
    exec(compile(src.replace(original, planted), "<mutant %s>" % fname, "exec"), ns)
    return ns[fname]


@pytest.mark.parametrize("name,fname,original,planted", PY_MUTANTS, ids=[m[0] for m in PY_MUTANTS])
def test_python_mutant_is_caught(name, fname, original, planted, monkeypatch):
    monkeypatch.setattr(orc, fname, _mutated_function(fname, original, planted))
    caught = _first_failing_pin()
    assert caught is not None, "no pin catches: " + name


def test_unmutated_oracle_passes_every_pin():
    assert _first_failing_pin() is None
