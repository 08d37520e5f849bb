"""The oracle's pins must catch plausible mistakes.

Each case copies ``oracle/lsb_oracle.c``, plants one mistake (a wrong bit
order, a dropped offset, a header in the wrong byte order, ...), builds the
copy with gcc and runs ``tests/test_oracle.py`` against it.  The run must
fail; a mutant that survives means a pin is missing.  Mistakes are planted in
the CPU oracle only.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lsb_oracle.c")

MUTANTS = {
    "stream_bits_lsb_first": ("(bytes[j / 8] >> (7 - (j % 8))) & 1u", "(bytes[j / 8] >> (j % 8)) & 1u"),
    "field_first_bit_lowest": ("v = (v << 1) | get_bit(stream, first + q);", "v |= get_bit(stream, first + q) << q;"),
    "header_little_endian": ("s[0] = (uint8_t)(len >> 24);", "s[0] = (uint8_t)len; s[3] = (uint8_t)(len >> 24); if (0)"),
    "partial_field_at_bottom": ("unsigned shift = (unsigned)k - nb;", "unsigned shift = 0;"),
    "partial_field_clears_all": ("stego[t] = (uint8_t)((cover[t] & ~mask & 0xFFu) | (v << shift));",
                                 "stego[t] = (uint8_t)((cover[t] & ~((1u << k) - 1u) & 0xFFu) | (v << shift));"),
    "extract_bit_reversed": ("unsigned bit = (stego[t] >> ((unsigned)k - 1 - q)) & 1u;", "unsigned bit = (stego[t] >> q) & 1u;"),
    "extract_drops_t0": ("uint64_t t = j / (uint64_t)k - t0;", "uint64_t t = j / (uint64_t)k;"),
    "embed_drops_t0": ("uint64_t first = (uint64_t)k * (t0 + t);", "uint64_t first = (uint64_t)k * t;"),
    "set_bit_lsb_first": ("bytes[j / 8] |= (uint8_t)(0x80u >> (j % 8));", "bytes[j / 8] |= (uint8_t)(0x01u << (j % 8));"),
    "capacity_off_by_one": ("uint64_t cap = room - 4;", "uint64_t cap = room - 3;"),
    "header_check_off_by_one": ("if (4 + (uint64_t)len > bits_to_bytes_floor(n, k))", "if (3 + (uint64_t)len > bits_to_bytes_floor(n, k))"),
    "tail_not_copied": ("stego[t] = cover[t]; /* past the stream: unchanged */", "stego[t] = 0;"),
    "paper_pixel_index_swapped": ("uint64_t at = plane_index(y, (uint32_t)(L * i + j), w, c, plane);\n                stego[at]",
                                  "uint64_t at = plane_index(y, (uint32_t)(4 * j + i), w, c, plane);\n                stego[at]"),
    "paper_pair_not_shifted": ("                v >>= 2 * i;\n", "                v >>= 0;\n"),
    "paper_rows_not_greedy": ("uint64_t L = remaining < w / 4 ? remaining : w / 4; /* size(B) */",
                              "uint64_t L = w / 4 < remaining ? w / 4 : remaining; if (y % 2) L = remaining < 1 ? remaining : 1;"),
    "paper_wrong_plane": ("return ((uint64_t)y * w + x) * c + plane;", "return ((uint64_t)y * w + x) * c;"),
    "paper_extract_no_shift": ("                v <<= 2 * i;\n", "                v <<= 0;\n"),
    "sse_abs_not_square": ("sum += (uint64_t)(d * d);", "sum += (uint64_t)(d < 0 ? -d : d);"),
    "psnr_peak_not_squared": ("return 10.0 * log10(255.0 * 255.0 / mse);", "return 10.0 * log10(255.0 / mse);"),
    "plane_index_dropped": ("        a[p] = cover[p * c + plane];\n", "        a[p] = cover[p * c];\n"),
    "buffer_check_missing": ("if ((uint64_t)len > out_cap)\n        return ORACLE_E_BUFFER;", "if (0)\n        return ORACLE_E_BUFFER;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation site not found: " + name
    mutant_c = tmp_path / "mutant.c"
    mutant_c.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-fPIC", "-shared",
                           "-I", os.path.join(ROOT, "oracle"),
                           "-o", str(lib), str(mutant_c), "-lm"])
    env = dict(os.environ, LSB_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle.py"),
                        os.path.join(ROOT, "tests", "test_oracle_paper.py"),
                        os.path.join(ROOT, "tests", "test_oracle_plane_psnr.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, "mutant %s survived every pin:\n%s" % (name, r.stdout[-2000:])
