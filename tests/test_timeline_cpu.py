"""The step-kernel timeline script's summary of its per-wavefront records (host logic only: the
records are made up here in the instrumented build's layout, 16 words per wavefront)."""
import pytest

from paper_1806_04960_amd import timeline


def record(entry, totals, entry_done, rows_done, located, own_end, exit_, strip, first, rows, steals):
    r = [entry, totals, entry_done, rows_done, located, own_end, exit_, strip, first, rows, steals]
    return r + [0] * (timeline.WORDS - len(r))


def test_summary_of_made_up_records():
    # 16 wavefronts; clock ticks are 10 ns; wavefront w starts at 100 w ticks (1 us apart)
    rec = []
    for w in range(16):
        t0 = 1000 + 100 * w
        rec.append(record(t0, t0 + 150, t0 + 300, t0 + 540, t0 + 700, t0 + 8000 + 10 * w, t0 + 9000 + 10 * w,
                          w % 4, 10 * w, 14 + (w % 3), w % 2))
    s = timeline.summarise(rec)
    assert s["wavefronts"] == 16
    # times in us from the first entry
    assert s["start"]["max"] == pytest.approx(15.0)
    assert s["launch_end"] == pytest.approx(15.0 + 90.0 + 1.5)
    assert s["locating_parts_median"]["strip_totals"] == pytest.approx(1.5)
    assert s["locating_parts_median"]["cut_search_and_strip_entry"] == pytest.approx(1.5)
    assert s["locating_parts_median"]["row_costs"] == pytest.approx(2.4)
    assert s["locating_parts_median"]["rest_of_locating"] == pytest.approx(1.6)
    assert s["own_range_rows_median"] == 15
    assert s["steals_total"] == 8
    # the latest own range is the last wavefront's, and so is the last exit
    assert s["latest_own_ranges"][0]["wavefront"] == 15
    assert s["latest_own_ranges"][0]["rows"] == [150, 150 + 14]
    assert s["latest_exits"][0]["wavefront"] == 15
    # per wavefront residue mod 8: wavefronts x and x + 8
    by = s["own_range_end_median_by_wavefront_mod_8"]
    assert len(by) == 8 and by[0] == pytest.approx(((80 + 0) + (80 + 8 + 0.8)) / 2)
