"""Host statistics over preconditioning levels (Tables I-III logic), on
hand-made per-configuration results whose table entries are counted by eye."""
import math

import pytest

from paper_0807_0264_amd import levels as LV


def res(level, R, v, blocks=10, Rs=None, plaq=600):
    return dict(level=level, R=R, R_smeared=Rs, vortices=v, blocks=blocks, plaquettes=plaq)


# three configurations, three levels "0", "4", "8"
CFG = [
    [res("0", 0.70, 30, 80), res("4", 0.72, 18, 110, 0.90), res("8", 0.73, 12, 130, 0.93)],
    [res("0", 0.71, 24, 70), res("4", 0.70, 24, 120, 0.91), res("8", 0.74, 20, 120, 0.94)],
    [res("0", 0.69, 36, 90), res("4", 0.71, 27, 100, 0.92), res("8", 0.70, 30, 140, 0.95)],
]


def test_table1_means_and_errors():
    t = LV.table1(CFG)
    assert [r["level"] for r in t] == ["0", "4", "8"]
    assert t[0]["blocks_mean"] == pytest.approx(80.0) and t[0]["blocks_std"] == pytest.approx(10.0)
    assert t[0]["R_smeared_mean"] is None
    assert t[1]["R_smeared_mean"] == pytest.approx(0.91)
    # standard error of (0.90, 0.91, 0.92): std 0.01 / sqrt(3)
    assert t[1]["R_smeared_sem"] == pytest.approx(0.01 / math.sqrt(3))
    assert t[2]["R_mean"] == pytest.approx((0.73 + 0.74 + 0.70) / 3)
    # vortex percentages at level 0: 5 %, 4 %, 6 %
    assert t[0]["vortex_pct_mean"] == pytest.approx(5.0) and t[0]["vortex_pct_sem"] == pytest.approx(1 / math.sqrt(3))


def test_transition_tables():
    tr = LV.transitions(CFG)
    assert tr["levels"] == ["0", "4", "8"] and tr["configurations"] == 3
    t2, t3 = tr["table2"], tr["table3"]
    assert all(t2[i][i] is None and t3[i][i] is None for i in range(3))
    # 0 -> 4: counts 30->18, 24->24, 36->27: two of three reduced
    assert t2[0][1] == pytest.approx(200 / 3)
    m, s = t2[1][0]  # reductions 40 % and 25 %
    assert m == pytest.approx(32.5) and s == pytest.approx(math.sqrt(2 * 7.5 ** 2))
    # 0 -> 8: 30->12, 24->20, 36->30: all reduced (60 %, 16.67 %, 16.67 %)
    assert t2[0][2] == pytest.approx(100.0)
    assert t2[2][0][0] == pytest.approx((60 + 50 / 3 + 50 / 3) / 3)
    # 4 -> 8: 18->12, 24->20, 27->30: two reduced
    assert t2[0 + 1][2] == pytest.approx(200 / 3)
    # higher maximum 0 -> 4: 0.72 > 0.70, 0.70 < 0.71, 0.71 > 0.69: two; both with fewer vortices
    assert t3[0][1] == pytest.approx(200 / 3) and t3[1][0] == pytest.approx(100.0)
    # 4 -> 8: 0.73 > 0.72, 0.74 > 0.70, 0.70 < 0.71: two; both with fewer vortices
    assert t3[1][2] == pytest.approx(200 / 3) and t3[2][1] == pytest.approx(100.0)
    # 0 -> 8: 0.73 > 0.70, 0.74 > 0.71, 0.70 > 0.69: all; all with fewer vortices
    assert t3[0][2] == pytest.approx(100.0) and t3[2][0] == pytest.approx(100.0)


def test_no_reduction_gives_none_and_higher_max_without_fewer_vortices():
    cfg = [[res("a", 0.70, 10), res("b", 0.75, 10)], [res("a", 0.70, 10), res("b", 0.75, 11)]]
    tr = LV.transitions(cfg)
    assert tr["table2"][0][1] == 0.0 and tr["table2"][1][0] is None
    assert tr["table3"][0][1] == 100.0 and tr["table3"][1][0] == 0.0


def test_paper_levels():
    assert [lv.n for lv in LV.PAPER_LEVELS] == [0, 4, 8, 12, 16, 20, 80]
    assert all(lv.rho == 0.1 and lv.eps == 1.0 for lv in LV.PAPER_LEVELS[:6])
    assert LV.PAPER_LEVELS[6].rho == 0.06 and LV.PAPER_LEVELS[6].eps == -0.25


def test_format_tables_renders():
    text = LV.format_tables(CFG)
    assert "vortex reduction" in text and "higher maximum" in text and "32.5+-10.6" in text


def test_tables_from_split_runs(tmp_path, capsys):
    """Configurations recorded one JSON line each, over two files (a split
    run, one configuration recorded twice), give the tables of the whole set."""
    import json
    a, b = tmp_path / "a.jsonl", tmp_path / "b.jsonl"
    a.write_text("".join(json.dumps(dict(config=c, levels=CFG[c])) + "\n" for c in (0, 1)))
    b.write_text("".join(json.dumps(dict(config=c, levels=CFG[c])) + "\n" for c in (1, 2)))
    LV.main(["--tables", str(a), str(b)])
    out = capsys.readouterr().out
    assert out.startswith("3 configurations") and LV.format_tables(CFG) in out
