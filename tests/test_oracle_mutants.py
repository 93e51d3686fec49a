"""The oracle's pins have teeth: plant plausible mistakes in a copy of
oracle.c (on the CPU), rebuild it, and check that the pin tests fail."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTANTS = {
    "delta_drops_min_delta": ("prev = prev + (uint64_t)min_delta + u;", "prev = prev + u;"),
    "rle_value_byte_count": ("uint64_t vb = (uint64_t)(w + 7) / 8;", "uint64_t vb = (uint64_t)w / 8;"),
    "bits_msb_first": ("v |= (uint64_t)((p[b >> 3] >> (b & 7)) & 1) << j;",
                       "v |= (uint64_t)((p[b >> 3] >> (7 - (b & 7))) & 1) << j;"),
    "snappy_copy_off_by_one": ("dst[op + k] = dst[op + k - off];", "dst[op + k] = dst[op + k - off + 1];"),
    "validity_inverted": ("if (!defs[i]) continue;", "if (defs[i]) continue;"),
    "snappy_copy1_offset_bits": ("off = ((uint64_t)(t >> 5) << 8) | src[r.pos];",
                                 "off = ((uint64_t)(t >> 5) << 7) | src[r.pos];"),
    "bitpacked_run_length": ("uint64_t nbytes = groups * (uint64_t)w;", "uint64_t nbytes = groups * (uint64_t)w + 1;"),
    "v2_values_offset": ("const uint8_t* cv = payload + h.rep_len + h.def_len;", "const uint8_t* cv = payload + h.rep_len;"),
    "dict_string_position": ("dict.spos[k] = q; dict.slen[k] = l;", "dict.spos[k] = q - 1; dict.slen[k] = l;"),
    "thrift_absolute_field_ids": ("if (delta) *id = *last_id + delta;", "if (delta) *id = delta;"),
    "delta_miniblock_width_index": ("int w = widths[m];", "int w = widths[0];"),
    "plain_width_int32_as_8": ("static int width_of(int type) { return type == 1 ? 4 : 8; }",
                               "static int width_of(int type) { return type == 1 ? 8 : 8; }"),
    "bss_row_major": ("v |= (uint64_t)p[(uint64_t)b * (uint64_t)count + (uint64_t)k] << (8 * b);",
                      "v |= (uint64_t)p[(uint64_t)k * (uint64_t)w + (uint64_t)b] << (8 * b);"),
    "dlba_lengths_skipped": ("  uint64_t q = (uint64_t)used;\n  for (int64_t k = 0; k < count; ++k) {\n    int32_t l",
                             "  uint64_t q = 0;\n  for (int64_t k = 0; k < count; ++k) {\n    int32_t l"),
    "dba_prefix_from_first_string": ("(*mat)[at + j] = (*mat)[pos[k - 1] + j];", "(*mat)[at + j] = (*mat)[pos[0] + j];"),
    "dba_suffix_offset": ("p[(uint64_t)used + spos[k] + j]", "p[spos[k] + j]"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    mut = tmp_path / "oracle_mut.c"
    mut.write_text(src.replace(old, new))
    so = tmp_path / "liboracle_mut.so"
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-shared", "-fPIC", str(mut), "-o", str(so)])
    env = dict(os.environ, PQ_ORACLE_SO=str(so), PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "tests/test_oracle_pins.py", "tests/test_oracle_files.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
