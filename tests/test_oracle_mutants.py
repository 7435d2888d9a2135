"""Plant plausible mistakes in copies of the oracle and check that the pin
battery catches every one (CPU only; the committed oracle is untouched)."""
import os
import subprocess
import sys

import pytest

from oracle import build as oracle_build
from tests import oracle_pins

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(os.path.dirname(oracle_build.__file__), "oracle.c")

MUTANTS = {
    "and_as_max": ("if (v < r) r = v;", "if (v > r) r = v;"),
    "or_as_min": ("if (v > r) r = v;", "if (v < r) r = v;"),
    "null_ignored": ("if (!c->valid) return 0;", "return 0;"),
    "between_open_hi": ("return from_bool(n->v1 <= x && x <= n->v2);",
                        "return from_bool(n->v1 <= x && x < n->v2);"),
    "not_unknown_to_false": ("return v == OC_T ? OC_F : (v == OC_F ? OC_T : OC_U);",
                             "return v == OC_T ? OC_F : (v == OC_F ? OC_T : OC_F);"),
    "lt_as_le": ("case CMP_LT: return from_bool(x < n->v1);",
                 "case CMP_LT: return from_bool(x <= n->v1);"),
    "in_drops_last": ("for (int64_t k = 0; k < n->cnt; k++)", "for (int64_t k = 1; k < n->cnt; k++)"),
    "codeset_inverted": ("return from_bool((w >> (x % 32)) & 1u);",
                         "return from_bool(!((w >> (x % 32)) & 1u));"),
    "int8_unsigned": ("case 1: return ((const int8_t*)c->data)[row];",
                      "case 1: return ((const uint8_t*)c->data)[row];"),
    "isunknown_as_isnull": ("return from_bool(eval(e, cols, e->children[n->off], row) == OC_U);",
                            "return from_bool(eval(e, cols, e->children[n->off], row) == OC_F);"),
    "limit_ge": ("if (c > max_rows) return 1;", "if (c >= max_rows) return 1;"),
    "rowid_shift": ("if (c < cap) out[c] = (uint32_t)i;", "if (c < cap) out[c] = (uint32_t)(i + 1);"),
    "star_skips_range": ("if (k < 0 || (uint64_t)k >= j->nbits[d]) return 0;",
                         "if (k < 0 || (uint64_t)k > j->nbits[d]) return 0;"),
    "keybitmap_offset": ("uint64_t b = (uint64_t)(k - key_min);", "uint64_t b = (uint64_t)k;"),
    "thread_split_gap": ("jobs[t].hi = nrows * (uint64_t)(t + 1) / (uint64_t)nt;",
                         "jobs[t].hi = nrows * (uint64_t)(t + 1) / (uint64_t)nt - (t + 1 < nt);"),
    "star_split_gap": ("nrows * (uint64_t)(t + 1) / (uint64_t)nt, 0};",
                       "nrows * (uint64_t)(t + 1) / (uint64_t)nt - (t + 1 < nt), 0};"),
    "rowids_split_gap": ("jobs[t].cap = cap;", "jobs[t].cap = cap;\n    if (t + 1 < nt) jobs[t].hi -= 1;"),
    "rowids_split_first": ("jobs[t].first = total;", "jobs[t].first = total + (t > 0);"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site of {name} not found"
    mutated = src.replace(old, new, 1)
    p = tmp_path / f"oracle_{name}.c"
    p.write_text(mutated)
    lib = oracle_build.build(src=str(p), out=str(tmp_path / f"liboracle_{name}.so"))
    # run the battery in a child: a mutant may also crash (which counts as caught)
    code = ("import sys; from tests import oracle_pins; "
            "f = oracle_pins.battery(sys.argv[1], quick=True); "
            "print(len(f), f[:3]); sys.exit(3 if f else 0)")
    r = subprocess.run([sys.executable, "-c", code, lib], cwd=ROOT, capture_output=True,
                       text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pin battery: {r.stdout}"
