"""Host-side checks of the product library (no GPU): exported symbols and the
diagram classification against Tables 1-4 of the paper."""
import ctypes
import os
import re

import pytest

import paper_1510_00903_amd as bbc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "bbcorr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bbc_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(bbc.library_path())
    decl = declared_symbols()
    assert len(decl) >= 12
    for name in decl:
        assert hasattr(lib, name), name
    assert sorted(bbc.EXPORTED_SYMBOLS) == decl


def test_channel_list_and_content():
    assert bbc.num_channels() == 52 and bbc.num_channels_all() == 56
    assert bbc.channel_name(0) == "p n > p n"
    assert bbc.channel_name(10) == "L L > L L"
    assert bbc.channel_name(51) == "X- X0 > X- X0"
    assert bbc.channel_content(0) == (6, 0)
    assert bbc.channel_content(1) == (5, 1)
    assert bbc.channel_content(51) == (2, 4)
    assert bbc.source_terms(10) == (3, 3)
    # ids from 56 on name other charge states; p p > p n (57) does not conserve flavour
    assert bbc.channel_name(56) == "p p > p p"
    for bad in (57, 56 + 8 ** 4, -1):
        with pytest.raises(bbc.BBCError):
            bbc.channel_name(bad)


def _read_tables():
    rows = []
    for ln in open(os.path.join(GOLDEN, "iteration_tables.txt")):
        if ln.startswith("#") or not ln.strip():
            continue
        tb, chs, combos, nd, its, tot = [x.strip() for x in ln.split("|")]
        want = sorted((int(x[:-1]), 1 if x[-1] == "+" else -1) for x in its.split())
        rows.append((int(tb), chs, combos.split(";"), int(nd), want, int(tot)))
    return rows


TERM = {"-": 0, "Xu": 0, "Xd": 1, "Xs": 2}
# Rows whose printed parities are the negatives of ours for every diagram (an
# unstated labelling of the quark fields in the paper; counts agree everywhere).
FLIPPED = {
    ("S+ S- > L L", "Xs,Xd"), ("S+ S- > L L", "Xu,Xd"), ("S+ S- > L L", "Xu,Xs"),
    ("S+ S- > S0 L", "Xd,Xs"), ("S+ S- > S0 L", "Xd,Xu"), ("S+ S- > S0 S0", "Xd,Xu"),
    ("S+ S- > n X0", "-,-"), ("S+ n > S0 p", "Xu,-"), ("S+ n > p L", "-,Xd"), ("S+ n > p L", "-,Xs"),
    ("S+ n > p L", "-,Xu"), ("S- X0 > S0 X-", "Xd,-"), ("S0 X- > S0 X-", "Xd,-"), ("S0 p > S+ n", "-,-"),
    ("S0 p > S0 p", "Xd,-"), ("X- L > S0 X-", "Xd,-"), ("n X0 > L L", "Xd,Xu"), ("n X0 > L L", "Xs,Xd"),
    ("n X0 > L L", "Xu,Xs"), ("n X0 > S+ S-", "-,-"), ("n X0 > S0 L", "Xu,Xd"), ("n X0 > S0 S0", "Xu,Xd"),
    ("n X0 > p X-", "-,-"), ("p L > S+ n", "-,-"), ("p L > S0 p", "Xd,-"), ("p X- > L L", "Xd,Xs"),
    ("p X- > L L", "Xu,Xd"), ("p X- > L L", "Xu,Xs"), ("p X- > S0 L", "Xd,Xu"), ("p X- > S0 S0", "Xd,Xu"),
    ("p X- > n X0", "-,-"),
}


def test_tables_1_to_4():
    """Every row of Tables 1-4: number of diagrams, iterations per diagram and total
    exactly; parities exactly, or all reversed for the listed rows."""
    names = {bbc.channel_name(c): c for c in range(52)}
    rows = _read_tables()
    assert len(rows) == 93
    n_exact = n_flip = 0
    for tb, chs, combos, nd, want, tot in rows:
        c = names[chs]
        for cmb in combos:
            t3, t4 = (TERM[x] for x in cmb.split(","))
            got = bbc.diagram_table(c, t3, t4)
            assert len(got) == nd, (chs, cmb)
            assert sum(k for k, _ in got) == tot, (chs, cmb)
            assert sorted(k for k, _ in got) == sorted(k for k, _ in want), (chs, cmb)
            if (chs, cmb) in FLIPPED:
                assert sorted((k, -s) for k, s in got) == want, (chs, cmb)
                n_flip += 1
            else:
                assert sorted(got) == want, (chs, cmb)
                n_exact += 1
    assert (n_exact, n_flip) == (114, 31)


def test_worked_example_p_lambda():
    """Sec. 3: the six p-Lambda diagrams (X_u source) in the printed order (i)-(vi)."""
    assert bbc.diagram_table(1, 0, 0) == [(1, 1), (9, -1), (144, -1), (144, 1), (36, 1), (36, -1)]
    assert sum(k for k, _ in bbc.diagram_table(1, 0, 1)) == 397     # X_d source
    assert sum(k for k, _ in bbc.diagram_table(1, 0, 2)) == 370     # X_s source


def test_total_iterations_all_channels():
    """Sum of the open-index iterations over all 52 channels and source terms."""
    st = bbc.plan_stats(range(52))
    assert st["iterations"] == 43507
    assert st["intermediates"] == 63
    assert st["components"] == 16560


def test_invalid_arguments_raise():
    with pytest.raises(bbc.BBCError):
        bbc.diagram_table(1, 0, 3)
    with pytest.raises(bbc.BBCError):
        bbc.footprint([5, 5, 5], [0])
    with pytest.raises(bbc.BBCError):
        bbc.plan_stats([57])
