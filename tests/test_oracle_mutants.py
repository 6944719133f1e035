"""Plant plausible mistakes in a copy of the oracle (on the CPU) and check
that the pins catch every one of them.  Each mutant runs in its own process,
so a mutant that reads out of bounds cannot take the test run down."""
import os
import subprocess
import sys

import pytest

from oracle import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    "overrun uses >=": ("if (n > avail_s) flags |= OR_SRC_OVERRUN;", "if (n >= avail_s) flags |= OR_SRC_OVERRUN;"),
    "A bit order reversed": ("(off & 63)) & 1u", "(63 - (off & 63))) & 1u"),
    "allocation end inclusive": ("(wide)p < (wide)s->abase[j] + s->asize[j]", "(wide)p <= (wide)s->abase[j] + s->asize[j]"),
    "only fully undefined bytes count": ("und = (vs != 0);", "und = (vs == 0xFF);"),
    "avail takes max": ("avail = avail_s < avail_d ? avail_s : avail_d;", "avail = avail_s > avail_d ? avail_s : avail_d;"),
    "propagate ignores source validity": ("uint8_t w = ok_s ? vs : 0xFF;", "uint8_t w = ok_s ? vs : 0;"),
    "first_bad ignores destination": ("(!ok_s || !ok_d || und)", "(!ok_s || und)"),
    "overlap off by one": ("if (s0 < d1 && d0 < s1)", "if (s0 < d1 && d0 + 1 < s1)"),
    "avail forgets the offset": ("avail_d = rd->abase[ad] + rd->asize[ad] - r->dst;", "avail_d = rd->asize[ad];"),
    "region end inclusive": ("x >= (wide)s->hb + s->hl", "x > (wide)s->hb + s->hl"),
    "dst unaddr never raised": ("if (dst_host && !ok_d) flags |= OR_DST_UNADDR;", ""),
    "device V index shifted": ("rd->av[as][r->src - rd->abase[as] + i]", "rd->av[as][r->src - rd->abase[as] + (i ? i - 1 : 0)]"),
    "propagation into overlapping copies": ("if (propagate && !overlap && ok_d)", "if (propagate && ok_d)"),
    "race ignores streams": ("if (eb != ea || streams[b] == streams[a]) continue;", "if (eb != ea) continue;"),
    "race ignores epochs": ("if (eb != ea || streams[b] == streams[a]) continue;",
                            "if (streams[b] == streams[a]) continue;"),
    "reads conflict with reads": ("if (meets(ra->src, ra->n, rb->dst, rb->n))",
                                  "if (meets(ra->src, ra->n, rb->dst, rb->n) || meets(ra->src, ra->n, rb->src, rb->n))"),
    "race ranges end inclusive": ("(wide)a < (wide)b + nb && (wide)b < (wide)a + na",
                                  "(wide)a <= (wide)b + nb && (wide)b <= (wide)a + na"),
    "race ranges wrap at 2^64": ("(wide)a < (wide)b + nb && (wide)b < (wide)a + na", "a < b + nb && b < a + na"),
    "race epochs cut to 15 bits": ("if (eb != ea || streams[b] == streams[a]) continue;",
                                   "if ((eb & 0x7FFFu) != (ea & 0x7FFFu) || streams[b] == streams[a]) continue;"),
    "race unchecked above 2^48": ("static int race_unchecked(const or_record *r) { return r->kind > OR_D2D; }",
                                  "static int race_unchecked(const or_record *r) { return r->kind > OR_D2D || "
                                  "(r->n && (wide)r->dst + r->n > ((wide)1 << 48)); }"),
    "unchecked records still meet": ("            if (race_unchecked(rb)) continue;\n", ""),
    "write-write conflicts missed": ("meets(ra->dst, ra->n, rb->dst, rb->n) || ", ""),
    "pointer one past the end rejected": ("            else if ((wide)p == end) past = (int64_t)j;\n", ""),
    "pointer one past wins over holding": ("int64_t j = hold >= 0 ? hold : past;", "int64_t j = past >= 0 ? past : hold;"),
    "pointer end inclusive": ("if ((wide)abase[j] <= p && (wide)p < end) hold = (int64_t)j;",
                              "if ((wide)abase[j] <= p && (wide)p <= end) hold = (int64_t)j;"),
    "pointer avail from base": ("out[t].avail = abase[j] + asize[j] - p;", "out[t].avail = asize[j];"),
    "zero length reports avail": ("if (n == 0) {\n        out->flags = 0; out->reserved = 0;\n        out->first_bad = OR_NONE; out->undef_bytes = 0; out->avail = 0;\n        return;\n    }", ""),
}


def test_unmodified_oracle_passes_battery(tmp_path):
    so = str(tmp_path / "lib_orig.so")
    oracle.build(out=so)
    r = subprocess.run([sys.executable, "-m", "tests.pin_battery", so], cwd=ROOT,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(oracle.SRC).read()
    assert src.count(old) == 1, name
    msrc = tmp_path / "oracle_mutant.c"
    msrc.write_text(src.replace(old, new))
    so = str(tmp_path / "lib_mutant.so")
    oracle.build(out=so, src=str(msrc))
    r = subprocess.run([sys.executable, "-m", "tests.pin_battery", so], cwd=ROOT,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0, f"mutant '{name}' survived the pins"
