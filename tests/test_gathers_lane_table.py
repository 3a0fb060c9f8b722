"""CPU check of the lane placement table of the 72-cell offset-gather
segments (csrc/gathers.hip, kPlace72): it places each of the 9 x 7 (cell
block, offset block) pairs exactly once, and under the LDS bank model of
16-byte reads (a wave is read in 4 passes of 16 lanes: lane bit 5 and the
parity of lane bits 2..4 pick the pass; a bank is a 16-byte chunk mod 16;
equal addresses never conflict) every pass reads U and V without conflicts,
for every nh the table serves (36 .. 41)."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GCX, BH, GM = 8, 12, 12


def _table():
    src = open(os.path.join(ROOT, "paper_2201_06914_amd", "csrc", "gathers.hip")).read()
    body = re.search(r"kPlace72\[4\]\[16\]\s*=\s*\{(.*?)\};", src, re.S).group(1)
    vals = [int(v, 16) for v in re.findall(r"0x([0-9A-Fa-f]{2})", body)]
    assert len(vals) == 64
    return [vals[16 * g:16 * g + 16] for g in range(4)]


def _pass_and_place(lane):
    q = (lane >> 2) & 7
    return 2 * (lane >> 5) + (bin(q).count("1") & 1), 4 * (q >> 1) + (lane & 3)


def test_table_places_every_pair_once():
    t = _table()
    pairs = [(e & 15, e >> 4) for row in t for e in row if e != 0xFF]
    assert sorted(pairs) == sorted((cb, hg) for cb in range(9) for hg in range(7))
    assert sum(e == 0xFF for row in t for e in row) == 1
    # lanes -> (pass, place) is a bijection onto 4 x 16
    assert len({_pass_and_place(l) for l in range(64)}) == 64


def test_table_reads_are_bank_conflict_free():
    t = _table()
    for nh in range(36, 42):
        sv = (4 - (2 * nh) % 4) % 4
        for field in ("U", "V"):
            for q in range(0, BH + GCX, 4):
                passes = {}
                for lane in range(64):
                    gp, k = _pass_and_place(lane)
                    e = t[gp][k]
                    if e == 0xFF:
                        continue
                    cb, hg = e & 15, e >> 4
                    base = (GCX * cb + hg * BH + GM if field == "U"
                            else GCX * cb - hg * BH - BH + 2 * nh + GM + sv)
                    chunk = (base + q) // 4
                    passes.setdefault(gp, {}).setdefault(chunk % 16, set()).add(chunk)
                for banks in passes.values():
                    assert all(len(a) == 1 for a in banks.values()), (nh, field, q)
