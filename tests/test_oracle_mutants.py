"""Planted mistakes in the oracle, on the CPU only.

Each mutant below is the oracle with one plausible mistake (a wrong operator, a dropped
term or stripe, a wrong index, bit order, stride or mask, a swapped operand).  Every mutant
must fail at least one of the oracle's own pins (the tests in ``test_oracle.py``, run
unchanged against the mutant), and the unmutated sources, built and loaded the same way,
must pass all of them.  This is what makes the pins evidence: they are not re-typings of
the oracle's formulas, and they catch the mistakes an implementation would plausibly make.
"""
import itertools
import os
import subprocess
import types

import pytest

import oracle
import test_oracle as pins
import test_oracle_mlp as mlp_pins

ORACLE_DIR = os.path.dirname(os.path.abspath(oracle.__file__))
C_SRC = open(os.path.join(ORACLE_DIR, "gf2ref.c")).read()
PY_SRC = open(os.path.join(ORACLE_DIR, "__init__.py")).read()
MLP_SRC = open(os.path.join(ORACLE_DIR, "mlp.py")).read()

# Mistakes in the C product (Sections 1 and 2): (text, replacement).
C_MUTANTS = {
    "addition as OR": ("acc[w] ^= brow[w];", "acc[w] |= brow[w];"),
    "short last stripe of k dropped": ("for (int64_t t = 0; t < k; ++t) {",
                                       "for (int64_t t = 0; t < (k & ~(int64_t)63); ++t) {"),
    "bits of A read most significant first": ("if ((arow[t >> 6] >> (t & 63)) & 1) {",
                                              "if ((arow[t >> 6] >> (63 - (t & 63))) & 1) {"),
    "row stride of B ignored": ("const uint64_t* brow = B + t * ldb;", "const uint64_t* brow = B + t * W;"),
    "row stride of A ignored": ("product_row(acc, A + i * lda, B, ldb, k, W);",
                                "product_row(acc, A + i * ((k + 63) >> 6), B, ldb, k, W);"),
    "padding of C not cleared": ("if (w == W - 1) v &= mask;", ";"),
    "accumulate mode ignored": ("crow[w] = accumulate ? (crow[w] ^ v) : v;", "crow[w] = v;"),
    "last row of C skipped": ("for (int64_t i = 0; i < m; ++i) {\n                product_row",
                              "for (int64_t i = 0; i < m - 1; ++i) {\n                product_row"),
    "padding mask one bit short": ("(((uint64_t)1 << r) - 1)", "(((uint64_t)1 << (r - 1)) - 1)"),
}

# Mistakes in the packed comparator the GPU checks use, the Four Russians steps (Section 3)
# and Algorithm 4 (Section 4).
PY_MUTANTS = {
    "comparator always equal": ("    return bool(np.array_equal(a, b))", "    return True"),
    "comparator masks the first word": ("        a[:, W - 1] &= mk\n        b[:, W - 1] &= mk",
                                        "        a[:, 0] &= mk\n        b[:, 0] &= mk"),
    "comparator skips the last word": ("    a = X[:, :W].copy()\n    b = Y[:, :W].copy()",
                                       "    a = X[:, :W - 1].copy()\n    b = Y[:, :W - 1].copy()"),
    "comparator reads the stride gap": ("    a = X[:, :W].copy()\n    b = Y[:, :W].copy()",
                                        "    a = X.copy()\n    b = Y.copy()"),
    "comparator mask one bit short": ("        mk = np.uint64((1 << r) - 1)", "        mk = np.uint64((1 << (r - 1)) - 1)"),
    "comparator skips the last row": ("    a = X[:, :W].copy()\n    b = Y[:, :W].copy()",
                                      "    a = X[:-1, :W].copy()\n    b = Y[:-1, :W].copy()"),
    "Gray code without the reflection": ("[[1] + c for c in reversed(code)]", "[[1] + c for c in code]"),
    "table row picked from the wrong end": ("src = r + pos[0]", "src = r + (kbits - 1 - pos[0])"),
    "ReadBits least significant first": ("        v = 2 * v + bit\n", "        v = v + (bit << b)\n"),
    "short last pass dropped": ("npass = -(-l // step) if l else 0", "npass = l // step"),
    "row blocking skips the last block": ("for s in range(0, m, block_rows)]", "for s in range(0, m - 1, block_rows)][:-1]"),
    "S1 with the wrong sign": ("S1 = sub(S0, A_NW)", "S1 = add(S0, A_NW)"),
    "T3 from the wrong operand": ("T3 = sub(T1, B_SW)", "T3 = sub(T0, B_SW)"),
    "P2 dropped from U4": ("U4 = add(U3, P2)", "U4 = U3"),
    "P5 with swapped operands": ("P5 = rec(S1, T1)", "P5 = rec(T1, S1) if S1.shape == T1.shape[::-1] else rec(S1, T0)"),
    "SE quadrant from U5": ("C[h:, :f], C[h:, f:] = U5, U6", "C[h:, :f], C[h:, f:] = U5, U5"),
    "peeled inner slice not added": ("Cm = ring.add(Cm, ring.base_mul(A[:me, le:], B[le:, :ne]))", "Cm = Cm"),
    "peeled last column block dropped": ("C[:me, ne:] = ring.base_mul(A[:me, :], B[:, ne:])", "pass"),
}

# Mistakes in the float64 schedule-model reference (forward, loss, chain rule, Adam).
MLP_MUTANTS = {
    "ReLU derivative dropped": ("g = (g @ W.T) * (pre[i - 1] > 0)", "g = g @ W.T"),
    "mask ignored in dL/dY": ("g = 2.0 * (Y - T) * M / cnt", "g = 2.0 * (Y - T) / cnt"),
    "dL/dY over all entries": ("g = 2.0 * (Y - T) * M / cnt", "g = 2.0 * (Y - T) * M / M.size"),
    "weight gradient halved": ("grads[2 * i] = acts[i].T @ g", "grads[2 * i] = 0.5 * (acts[i].T @ g)"),
    "bias gradient from the first row only": ("grads[2 * i + 1] = g.sum(axis=0)", "grads[2 * i + 1] = g[0].copy()"),
    "Adam without bias correction": ("mhat = mi / (1 - beta1 ** t)", "mhat = mi"),
    "Adam second moment not squared": ("vi = beta2 * vi + (1 - beta2) * g * g", "vi = beta2 * vi + (1 - beta2) * np.abs(g)"),
}


def build_lib(c_src, where):
    os.makedirs(where, exist_ok=True)
    src = os.path.join(where, "gf2ref.c")
    with open(src, "w") as f:
        f.write(c_src)
    lib = os.path.join(where, "liboracle_gf2.so")
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", src, "-o", lib], check=True)
    return where


def load_module(py_src, libdir, name):
    mod = types.ModuleType(name)
    mod.__file__ = os.path.join(libdir, "__init__.py")
    exec(compile(py_src, mod.__file__, "exec"), mod.__dict__)
    mod._HERE = libdir
    mod._LIB = None
    return mod


# The one pin that takes seconds runs last, so a mutant is usually caught before it.
SLOW_LAST = ("test_mul_matches_bruteforce_and_numpy_up_to_1024",)


def pin_cases(module):
    """Every test of a pin module with every parameter set it is run with."""
    for name in sorted(dir(module), key=lambda nm: (nm in SLOW_LAST, nm)):
        fn = getattr(module, name)
        if not (name.startswith("test_") and callable(fn)):
            continue
        grids = [m for m in getattr(fn, "pytestmark", []) if m.name == "parametrize"]
        if not grids:
            yield name, fn, {}
            continue
        axes = []
        for mk in grids:
            names = [s.strip() for s in mk.args[0].split(",")] if isinstance(mk.args[0], str) else list(mk.args[0])
            vals = [v if len(names) > 1 else (v,) for v in mk.args[1]]
            axes.append([dict(zip(names, v)) for v in vals])
        for combo in itertools.product(*axes):
            kw = {}
            for d in combo:
                kw.update(d)
            yield name, fn, kw


def run_pins(mod, monkeypatch, stop_at_first, module=pins, attr="oracle"):
    monkeypatch.setattr(module, attr, mod)
    failed = []
    for name, fn, kw in pin_cases(module):
        try:
            fn(**kw)
        except Exception as e:       # an assertion, or the oracle refusing its own inputs
            failed.append(f"{name}{kw or ''}: {type(e).__name__}")
            if stop_at_first:
                break
    monkeypatch.undo()
    return failed


@pytest.fixture(scope="module")
def good_libdir(tmp_path_factory):
    return build_lib(C_SRC, str(tmp_path_factory.mktemp("oracle_good")))


def test_unmutated_oracle_passes_every_pin(good_libdir, monkeypatch):
    mod = load_module(PY_SRC, good_libdir, "oracle_unmutated")
    assert run_pins(mod, monkeypatch, stop_at_first=False) == []
    mlp = load_module(MLP_SRC, good_libdir, "mlp_unmutated")
    assert run_pins(mlp, monkeypatch, stop_at_first=False, module=mlp_pins, attr="mlp") == []


@pytest.mark.parametrize("mutant", sorted(C_MUTANTS))
def test_c_mutant_fails_a_pin(mutant, tmp_path, monkeypatch):
    old, new = C_MUTANTS[mutant]
    assert C_SRC.count(old) == 1, f"mutation site of {mutant!r} not found exactly once"
    libdir = build_lib(C_SRC.replace(old, new), str(tmp_path))
    mod = load_module(PY_SRC, libdir, "oracle_mutant")
    failed = run_pins(mod, monkeypatch, stop_at_first=True)
    assert failed, f"no pin catches the mutant {mutant!r}"
    print(mutant, "->", failed[0])


@pytest.mark.parametrize("mutant", sorted(PY_MUTANTS))
def test_python_mutant_fails_a_pin(mutant, good_libdir, monkeypatch):
    old, new = PY_MUTANTS[mutant]
    assert PY_SRC.count(old) == 1, f"mutation site of {mutant!r} not found exactly once"
    mod = load_module(PY_SRC.replace(old, new), good_libdir, "oracle_mutant")
    failed = run_pins(mod, monkeypatch, stop_at_first=True)
    assert failed, f"no pin catches the mutant {mutant!r}"
    print(mutant, "->", failed[0])


@pytest.mark.parametrize("mutant", sorted(MLP_MUTANTS))
def test_mlp_mutant_fails_a_pin(mutant, good_libdir, monkeypatch):
    old, new = MLP_MUTANTS[mutant]
    assert MLP_SRC.count(old) == 1, f"mutation site of {mutant!r} not found exactly once"
    mod = load_module(MLP_SRC.replace(old, new), good_libdir, "mlp_mutant")
    failed = run_pins(mod, monkeypatch, stop_at_first=True, module=mlp_pins, attr="mlp")
    assert failed, f"no pin catches the mutant {mutant!r}"
    print(mutant, "->", failed[0])
