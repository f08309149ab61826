"""Planted mistakes in copies of the oracle must each fail a pin.

Each mutant is the oracle source with one plausible slip (a dropped term, a
wrong identity, an off-by-one bound, a swapped comparison, a wrong shift,
a wrong offset) compiled on the CPU; the real oracle is never modified.
"""
import os

import pytest

import oracle
import oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "lscan_oracle.c")

# (name, text to replace, replacement, which occurrence: 0 = first)
MUTANTS = [
    ("loop_drops_last", "for (int64_t j = 0; j < n; ++j) {", "for (int64_t j = 0; j + 1 < n; ++j) {", 0),
    ("i64_loop_drops_last", "for (int64_t j = 0; j < n; ++j) {", "for (int64_t j = 0; j + 1 < n; ++j) {", 1),
    ("excl_after_update", "if (exclusive) y[j] = acc;\n        if (op == OR_ADD)\n            acc = (int32_t)",
     "if (op == OR_ADD)\n            acc = (int32_t)", 0),
    ("max_identity_zero", "(op == OR_MAX) ? INT32_MIN : INT32_MAX", "(op == OR_MAX) ? 0 : INT32_MAX", 0),
    ("min_identity_zero", "(op == OR_MAX) ? INT64_MIN : INT64_MAX", "(op == OR_MAX) ? INT64_MIN : 0", 0),
    ("max_compare_swapped", "acc = (v > acc) ? v : acc;", "acc = (v < acc) ? v : acc;", 0),
    ("min_compare_swapped", "acc = (v < acc) ? v : acc;", "acc = (v > acc) ? v : acc;", 1),
    ("add_becomes_sub", "acc = (int32_t)((uint32_t)acc + (uint32_t)v);", "acc = (int32_t)((uint32_t)acc - (uint32_t)v);", 0),
    ("neumaier_dropped", "*c += (*s - t) + v;", "*c += 0.0;", 0),
    ("neumaier_branch_swapped", "*c += (v - t) + *s;", "*c += (*s - t) + v;", 0),
    ("absum_signed", "a += fabs(v);", "a += v;", 0),
    ("zero_order_ignored", "return signbit(a) && !signbit(b);", "return 0;", 0),
    ("zero_order_reversed", "return signbit(a) && !signbit(b);", "return !signbit(a) && signbit(b);", 0),
    ("bf16_shift", "uint32_t bits = (uint32_t)h << 16;", "uint32_t bits = (uint32_t)h << 15;", 0),
    ("float_max_identity", "float acc = (op == OR_MAX) ? -INFINITY : INFINITY;", "float acc = (op == OR_MAX) ? 0.0f : INFINITY;", 0),
    ("seg_offset_bytes", "(const char *)x + lo * isz", "(const char *)x + lo", 0),
    ("seg_len_short", "hi - lo, dtype, op,", "hi - lo - (hi > lo), dtype, op,", 0),
    ("compact_keep_inverted", "take = keep[i] != 0;", "take = keep[i] == 0;", 0),
    ("compact_last_dropped", "for (int64_t i = 0; i < n; ++i) {\n        const unsigned char *e", "for (int64_t i = 0; i + 1 < n; ++i) {\n        const unsigned char *e", 0),
    ("compact_first_byte_only", "for (int b = 0; b < elem_size; ++b) take |= e[b] != 0;", "take = e[0] != 0;", 0),
    ("compact_stride_one", "const unsigned char *e = src + i * elem_size;", "const unsigned char *e = src + i;", 0),
    ("compact_dst_not_advanced", "memcpy(dst + count * elem_size, e, (size_t)elem_size);", "memcpy(dst, e, (size_t)elem_size);", 0),
    ("radix_block_major", "out[d * m + i / block_items] += 1;", "out[(i / block_items) * nd + d] += 1;", 0),
    ("radix_inclusive", "out[i] = acc;\n        acc += c;", "acc += c;\n        out[i] = acc;", 0),
    ("radix_shift_ignored", "int64_t d = (int64_t)((k >> shift) & mask);", "int64_t d = (int64_t)(k & mask);", 0),
    ("radix_key_truncated", ": ((const uint64_t *)keys)[i];", ": (uint64_t)((const uint32_t *)keys)[i];", 0),
    ("argscan_ties_to_last", "better = want_max ? (v > b) : (v < b);\n        } else if (dtype == OR_I64)", "better = want_max ? (v >= b) : (v <= b);\n        } else if (dtype == OR_I64)", 0),
    ("argscan_i64_inverted", "better = want_max ? (v > b) : (v < b);\n        } else {", "better = want_max ? (v < b) : (v > b);\n        } else {", 0),
    ("argscan_float_zero_order", "better = want_max ? total_less(b, v) : total_less(v, b);", "better = want_max ? (v > b) : (v < b);", 0),
    ("argscan_excl_after", "if (exclusive) y[j] = best;\n        int better;", "int better;", 0),
    ("affine_swapped_composition", "pb = a * pb + b; /* apply the prefix, then map j */", "pb = pa * b + pb;", 0),
    ("affine_identity_zero", "uint32_t pa = 1u, pb = 0u; /* the identity map */", "uint32_t pa = 0u, pb = 0u;", 0),
    ("affine_dropped_offset", "pb = a * pb + b; /* apply the prefix, then map j */", "pb = a * pb;", 0),
    ("bfs_level_not_incremented", "level[v] = level[u] + 1;", "level[v] = level[u];", 0),
    ("bfs_stack_order", "int32_t u = queue[head++];", "int32_t u = queue[--tail];", 0),
    ("bfs_source_level_one", "level[src] = 0;", "level[src] = 1;", 0),
    ("bfs_first_edge_skipped", "for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {", "for (int64_t e = row_ptr[u] + 1; e < row_ptr[u + 1]; ++e) {", 0),
    ("excl_float_stale_abs", "if (absum) absum[j] = a;\n        }\n        neumaier_add(&s, &c, v);\n        a += fabs(v);\n        if (!exclusive) {\n            y64[j] = s + c;",
     "if (absum) absum[j] = a + fabs(v);\n        }\n        neumaier_add(&s, &c, v);\n        a += fabs(v);\n        if (!exclusive) {\n            y64[j] = s + c;", 0),
]


def _replace_nth(text, old, new, nth):
    idx = -1
    for _ in range(nth + 1):
        idx = text.find(old, idx + 1)
        if idx < 0:
            raise AssertionError(f"mutation anchor not found: {old!r} #{nth}")
    return text[:idx] + new + text[idx + len(old):]


def test_real_oracle_passes_every_pin():
    oracle.build(force=False)
    assert pins.failing_checks(oracle.default()) == []


@pytest.mark.parametrize("name,old,new,nth", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, old, new, nth):
    src = open(SRC).read()
    mutated = _replace_nth(src, old, new, nth)
    assert mutated != src
    c_path = tmp_path / f"{name}.c"
    c_path.write_text(mutated)
    so = oracle.compile_library(str(c_path), str(tmp_path / f"lib{name}.so"))
    failures = pins.failing_checks(oracle.Oracle(so))
    assert failures, f"mutant {name} passed every pin"
