"""The C ABI without a GPU: the library loads, exports every function include/gf2.h declares,
and rejects bad arguments with the documented status before touching a device."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_0811_1714_amd as g

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if not h.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for mt in re.finditer(r"\b(gf2_[a-z0-9_]+)\s*\(", text):
            names.add(mt.group(1))
    return sorted(names)


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert "gf2_mul" in names and "gf2_addmul" in names
    out = subprocess.run(["nm", "-D", "--defined-only", g.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    L = g.lib()
    for n in names:
        assert hasattr(L, n)


P = ctypes.c_void_p


def call(m, k, n, C=0x10000, ldc=2, A=0x20000, lda=2, B=0x30000, ldb=2, fn="gf2_mul"):
    return getattr(g.lib(), fn)(P(C), ldc, P(A), lda, P(B), ldb, m, k, n, None)


@pytest.mark.parametrize("fn", ["gf2_mul", "gf2_addmul"])
def test_validation_codes(fn):
    INV, ALIAS, UNSUP = 1, 2, 6
    assert call(-1, 5, 5, fn=fn) == INV
    assert call(5, -1, 5, fn=fn) == INV
    assert call(5, 5, -1, fn=fn) == INV
    assert call(5, 100, 5, lda=1, fn=fn) == INV          # lda < ceil(k/64)
    assert call(5, 5, 200, ldb=3, ldc=4, fn=fn) == INV   # ldb < ceil(n/64)
    assert call(5, 5, 200, ldb=4, ldc=3, fn=fn) == INV   # ldc < ceil(n/64)
    assert call(5, 5, 5, C=0, fn=fn) == INV
    assert call(5, 5, 5, A=0, fn=fn) == INV
    assert call(5, 5, 5, B=0, fn=fn) == INV
    assert call(5, 5, 5, C=0x10004, fn=fn) == INV        # misaligned
    assert call(5, 5, 5, A=0x20001, fn=fn) == INV
    assert call(5, 5, 5, C=0x20008, fn=fn) == ALIAS      # C inside A
    assert call(5, 5, 5, C=0x30000, fn=fn) == ALIAS      # C == B
    assert call(1 << 31, 5, 5, fn=fn) == UNSUP
    assert call(5, 5, 5, ldc=1 << 22, fn=fn) == UNSUP
    assert g.last_error() != ""
    # empty products are no-ops that never touch the device
    assert call(0, 5, 5, fn=fn) == 0
    assert call(5, 5, 0, fn=fn) == 0


def test_schedule_validation():
    L = g.lib()
    bad = [g.Schedule(9, 0, 0, 1), g.Schedule(g.KERNEL_M4RM, 99, 0, 1), g.Schedule(g.KERNEL_M4RM, 0, -1, 1),
           g.Schedule(g.KERNEL_M4RM, 0, 0, 1000), g.Schedule(g.KERNEL_M4RM, 0, 512, 1, 2)]
    for s in bad:
        r = L.gf2_mul_sched(P(0x10000), 2, P(0x20000), 2, P(0x30000), 2, 5, 5, 5, 0, ctypes.byref(s), None)
        assert r in (1, 6), (s, r)


def test_status_strings():
    L = g.lib()
    for code, name in g.STATUS.items():
        assert L.gf2_status_string(code).decode() == name


def test_workspace_sizing_matches_plan():
    # Strassen-Winograd, one level on 1024^3: 4 S (512x8 words), 4 T (512x8), 7 P (512x8) buffers.
    s = g.Schedule(g.KERNEL_M4RM, 0, 512, 1)
    assert g.workspace_bytes(1024, 1024, 1024, s) == 15 * 512 * 8 * 8
    assert g.workspace_bytes(1024, 1024, 1024, g.Schedule(g.KERNEL_M4RM, 0, 0, 1)) == 0


def test_batch_validation_without_device():
    L = g.lib()

    def prob(C, A, B, m=5, k=5, n=5, ld=1, sched=-1):
        return g.Problem(A, B, C, m, k, n, ld, ld, ld, 0, sched)

    def run(probs):
        arr = (g.Problem * len(probs))(*probs)
        h = ctypes.c_void_p(0)
        return L.gf2_batch_plan_create(arr, len(probs), ctypes.byref(h))

    assert run([prob(0x10000, 0x20000, 0x30000, m=-1)]) == 1
    assert run([prob(0x10000, 0x20000, 0x30000, sched=99)]) == 1
    assert run([prob(0x10000, 0x20000, 0x30000), prob(0x10000 + 16, 0x40000, 0x50000)]) == 2   # C's overlap
    assert run([prob(0x10000, 0x20000, 0x30000), prob(0x60000, 0x10000, 0x50000)]) == 2        # C is another's A
    assert L.gf2_mul_batched(None, 3, None) == 1
    assert L.gf2_num_candidates() >= 8


def test_schedule_struct_layout():
    """gf2_schedule is seven int32 fields (kernel, variant, cutoff, splitk, odd, kappa, memory)."""
    import ctypes
    import paper_0811_1714_amd as g
    assert ctypes.sizeof(g.Schedule) == 28
    assert [f[0] for f in g.Schedule._fields_] == ["kernel", "variant", "cutoff", "splitk", "odd", "kappa", "memory"]
    assert (g.ODD_PAD, g.ODD_PEEL, g.MEM_FAST, g.MEM_LOW) == (0, 1, 0, 1)


def test_two_temporary_workspace():
    """Section 4's memory-efficient schedule at the top level keeps two temporaries, X (m/2 x
    max(k, n)/2) and Y (k/2 x n/2), plus the breadth-first workspace of one of its products."""
    import paper_0811_1714_amd as g
    low = g.Schedule(g.KERNEL_M4RM, 1, 256, 1, 0, 0, g.MEM_LOW)
    fast = g.Schedule(g.KERNEL_M4RM, 1, 256, 1, 0, 0, g.MEM_FAST)
    # 1024^3: X, Y 512 x 8 words each; a 512^3 product one level down: 15 quadrants of 256 x 4 words.
    assert g.workspace_bytes(1024, 1024, 1024, low) == (2 * 512 * 8 + 15 * 256 * 4) * 8
    # Breadth-first, two exact levels: the passes of both levels are fused, so the top node keeps
    # only its S and T (8 quadrants of 512 x 8 words); each child its 15 of 256 x 4.
    assert g.workspace_bytes(1024, 1024, 1024, fast) == (8 * 512 * 8 + 7 * 15 * 256 * 4) * 8
    # Not exact (1000 columns): the top node's P0..P6 are kept too.
    assert g.workspace_bytes(1024, 1024, 1000, fast) > g.workspace_bytes(1024, 1024, 1024, fast)
    # 32768^3 over 8192-row leaves: 1096 MiB breadth-first, 184 MiB with two temporaries.
    big_low = g.Schedule(g.KERNEL_M4RM, 16, 8192, 1, 0, 0, g.MEM_LOW)
    big_fast = g.Schedule(g.KERNEL_M4RM, 16, 8192, 1, 0, 0, g.MEM_FAST)
    assert g.workspace_bytes(32768, 32768, 32768, big_fast) == 1096 << 20
    assert g.workspace_bytes(32768, 32768, 32768, big_low) == 184 << 20
    # Odd rows: the two-temporary form does not apply, the figure is the breadth-first one.
    assert g.workspace_bytes(1025, 1024, 1024, low) == g.workspace_bytes(1025, 1024, 1024, fast)
    try:
        g.resolve_schedule(100, 100, 100, g.Schedule(g.KERNEL_M4RM, 1, 0, 1, 0, 0, 2))
    except g.GF2Error as e:
        assert e.status == 1
    else:
        raise AssertionError("workspace plan 2 accepted")


def test_table_width_validation_and_workspace():
    """kappa 0 means 8; 4..7 only on the tiles of at most 1024 rows (the others, and widths outside
    4..8, are refused); a narrow table's workspace holds A's index bytes, one per kappa bits of k,
    rounded up to whole words per row, 256-byte aligned per product."""
    import paper_0811_1714_amd as g
    narrow = {1, 2, 3, 4, 12, 13, 18, 19, 20}
    assert g.resolve_schedule(1000, 1000, 1000, g.Schedule(g.KERNEL_M4RM, 2, 0, 1)).kappa == 8
    for v in range(g.kernel_variants(g.KERNEL_M4RM)):
        for kappa in (4, 5, 6, 7, 8):
            s = g.Schedule(g.KERNEL_M4RM, v, 0, 1, 0, kappa)
            if kappa == 8 or v in narrow:
                assert g.resolve_schedule(1000, 1000, 1000, s).kappa == kappa
            else:
                try:
                    g.resolve_schedule(1000, 1000, 1000, s)
                except g.GF2Error as e:
                    assert e.status == 6, (v, kappa)
                else:
                    raise AssertionError(f"variant {v} accepted {kappa}-bit tables")
    for bad in (1, 3, 9, -1):
        try:
            g.resolve_schedule(100, 100, 100, g.Schedule(g.KERNEL_M4RM, 2, 0, 1, 0, bad))
        except g.GF2Error as e:
            assert e.status == 1
        else:
            raise AssertionError(f"table width {bad} accepted")
    # 1000 x 1000 at 6 bits: 167 index bytes -> 21 words per row; 21000 words, aligned to 32.
    assert g.workspace_bytes(1000, 1000, 1000, g.Schedule(g.KERNEL_M4RM, 2, 0, 1, 0, 6)) == 21024 * 8
    # k in four slices of 4 words: each slice's 256 bits give 52 bytes at 5 bits -> 7 words per row.
    assert g.workspace_bytes(100, 1024, 500, g.Schedule(g.KERNEL_M4RM, 2, 0, 4, 0, 5)) == 4 * 704 * 8


def test_peeling_workspace_is_sized_for_the_aligned_core():
    """Peeling recurses on the largest part with even rows and k, n multiples of 128, so a
    2^10+1 product needs the temporaries of the 1024 core's node (quadrants of 512 x 8 words)."""
    import paper_0811_1714_amd as g
    peel = g.workspace_bytes(1025, 1025, 1025, g.Schedule(g.KERNEL_M4RM, 0, 512, 1, g.ODD_PEEL))
    core = g.workspace_bytes(1024, 1024, 1024, g.Schedule(g.KERNEL_M4RM, 0, 512, 1, g.ODD_PAD))
    pad = g.workspace_bytes(1025, 1025, 1025, g.Schedule(g.KERNEL_M4RM, 0, 512, 1, g.ODD_PAD))
    assert peel == core == 15 * 512 * 8 * 8
    assert pad > peel     # padding splits at 513 rows / 9 words



def test_resolve_schedule_without_gpu():
    """gf2_resolve_schedule reports what a call would run: the cost-model default for large
    products (no GPU needed under the fixed policy), requested fields kept, bad input refused."""
    import paper_0811_1714_amd as g
    s = g.resolve_schedule(32768, 32768, 32768)
    assert s.kernel == g.KERNEL_M4RM and s.cutoff > 0 and s.splitk == 1     # Strassen-Winograd over M4RM
    v = g.resolve_schedule(32768, 32768, 1)
    assert v.kernel == g.KERNEL_CUBIC and v.cutoff == 0                      # matrix-vector: streamed popcount
    w = g.resolve_schedule(32768, 32768, 64)
    assert w.kernel == g.KERNEL_M4RM and w.cutoff == 0 and w.splitk > 1     # one-word tiles, k split
    assert g.kernel_variants(g.KERNEL_M4RM) > w.variant >= 0
    req = g.Schedule(g.KERNEL_MFMA, 0, 4096, 1, g.ODD_PEEL)
    r = g.resolve_schedule(10000, 10000, 10000, req)
    assert (r.kernel, r.variant, r.cutoff, r.splitk, r.odd) == (g.KERNEL_MFMA, 0, 4096, 1, g.ODD_PEEL)
    for bad in ((-1, 5, 5, None), (5, 5, 5, g.Schedule(g.KERNEL_M4RM, 999, 0, 1))):
        try:
            g.resolve_schedule(*bad)
        except g.GF2Error as e:
            assert e.status == 1
        else:
            raise AssertionError(f"{bad} accepted")


def test_autotune_candidates_validation():
    """The partial re-timing call refuses an out-of-range candidate index, a negative count, a
    missing list and a bad density with GF2_ERR_INVALID_ARG before any device work."""
    import ctypes
    import paper_0811_1714_amd as g
    S = g.num_candidates()
    for cands, dens in (([S], 0.5), ([-1], 0.5), ([0, S + 3], 0.5), ([1], 1.5), ([1], -0.1)):
        with pytest.raises(g.GF2Error) as ei:
            g.autotune_candidates(100, 100, 100, cands, density=dens)
        assert ei.value.status == 1, (cands, dens)
    ms = (ctypes.c_float * S)()
    assert g.lib().gf2_autotune_candidates(100, 100, 100, 0.5, 1, 1, None, 1, ms, None) == 1
    assert g.lib().gf2_autotune_candidates(100, 100, 100, 0.5, 1, 1, None, -1, ms, None) == 1


def test_autotune_cache_failure_paths(tmp_path):
    """Corrupt, truncated and missing autotune cache files are refused with GF2_ERR_INVALID_ARG and
    leave the cache as it was; a well-formed file loads, and saving it back gives the same entries."""
    import paper_0811_1714_amd as g
    S = g.num_candidates()
    g.autotune_clear()
    good = tmp_path / "good.txt"
    row = " ".join(str(0.5 + c) for c in range(S))
    good.write_text(f"20 20 20 {row}\n22 18 14 {row}\n")
    g.autotune_load(str(good))
    saved = tmp_path / "saved.txt"
    g.autotune_save(str(saved))
    lines = sorted(saved.read_text().split("\n"))
    assert [ln.split()[:3] for ln in lines if ln] == [["20", "20", "20"], ["22", "18", "14"]]
    assert all(len(ln.split()) == 3 + S for ln in lines if ln)
    cases = {
        "truncated": f"20 20 20 {row}\n24 24 24 " + " ".join(["1.0"] * (S - 1)) + "\n",
        "not numbers": f"20 20 20 {row}\nx y z {row}\n",
        "garbage value": f"26 26 26 " + " ".join(["1.0"] * (S - 1)) + " nan?\n",
        "binary": "\x00\x01\x02\xff\xfe",
    }
    for name, text in cases.items():
        bad = tmp_path / f"{name}.txt"
        bad.write_bytes(text.encode("latin-1"))
        with pytest.raises(g.GF2Error) as ei:
            g.autotune_load(str(bad))
        assert ei.value.status == 1, name
        after = tmp_path / f"after_{name}.txt"
        g.autotune_save(str(after))
        assert sorted(after.read_text().split("\n")) == lines, f"{name}: cache changed by a refused load"
    with pytest.raises(g.GF2Error) as ei:
        g.autotune_load(str(tmp_path / "missing.txt"))
    assert ei.value.status == 1
    with pytest.raises(g.GF2Error) as ei:
        g.autotune_save(str(tmp_path / "no_such_dir" / "x.txt"))
    assert ei.value.status == 1
    assert g.lib().gf2_autotune_load(None) == 1
    g.autotune_clear()


def test_lds_probe_argument_errors():
    L = g.lib()
    d = ctypes.c_double(0)
    assert L.gf2_lds_probe(2, 1, 1, P(0x10000), ctypes.byref(d), None) == 1
    assert L.gf2_lds_probe(0, 0, 1, P(0x10000), ctypes.byref(d), None) == 1
    assert L.gf2_lds_probe(0, 1, 0, P(0x10000), ctypes.byref(d), None) == 1
    assert L.gf2_lds_probe(1, 1, 1, P(0), ctypes.byref(d), None) == 1
