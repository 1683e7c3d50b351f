"""The Python binding's ctypes structures against the C headers, field by
field: a small C program compiled with gcc prints sizeof and offsetof of
every ABI struct (include/*.h) and of the oracle's structs, and each must
equal its ctypes counterpart."""
import ctypes
import json
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (C struct, Python class path, fields)
LIB_STRUCTS = [
    ("plas_sort_params", "SortParams"), ("plas_sort_stats", "SortStats"), ("plas_level_stat", "LevelStat"),
    ("plas_sort_checkpoint", "Checkpoint"), ("plas_batch_item", "BatchItem"), ("plas_tune_entry", "TuneEntry"),
    ("plas_batch_config", "BatchConfig"), ("plas_batch_stats", "BatchStats"),
]
ORACLE_STRUCTS = [
    ("plas_ref_params", "_Params"), ("plas_ref_result", "_Result"), ("plas_ref_level", "_Level"),
    ("plas_ref_state", "State"),
]


def _c_layout(tmp_path, header_includes, structs):
    lines = ["#include <stddef.h>", "#include <stdio.h>"] + [f'#include "{h}"' for h in header_includes]
    lines.append("int main(void) {")
    lines.append('  printf("{");')
    first = True
    for cname, fields in structs:
        parts = [f'\\"size\\": %zu'] + [f'\\"{f}\\": %zu' for f in fields]
        args = [f"sizeof({cname})"] + [f"offsetof({cname}, {f})" for f in fields]
        sep = "" if first else ", "
        first = False
        lines.append(f'  printf("{sep}\\"{cname}\\": {{{", ".join(parts)}}}", {", ".join(args)});')
    lines.append('  printf("}\\n");')
    lines.append("  return 0;\n}")
    src = tmp_path / "layout.c"
    exe = tmp_path / "layout"
    src.write_text("\n".join(lines))
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-I",
                           os.path.join(ROOT, "oracle"), str(src), "-o", str(exe)])
    return json.loads(subprocess.check_output([str(exe)]).decode())


def _check(module, pairs, tmp_path, headers):
    structs = [(c, [f[0] for f in getattr(module, py)._fields_]) for c, py in pairs]
    layout = _c_layout(tmp_path, headers, structs)
    for c, py in pairs:
        cls = getattr(module, py)
        assert layout[c]["size"] == ctypes.sizeof(cls), c
        for name, _ in cls._fields_:
            assert layout[c][name] == getattr(cls, name).offset, (c, name)


def test_library_structs_match_the_headers(tmp_path):
    import paper_2312_13299_amd as plas
    _check(plas, LIB_STRUCTS, tmp_path, ["plas.h", "plas_batch.h", "plas_stages.h"])


def test_oracle_structs_match_its_header(tmp_path):
    import oracle
    _check(oracle, ORACLE_STRUCTS, tmp_path, ["plas_oracle.h"])


def test_binding_abi_version_matches_the_header():
    import re
    import paper_2312_13299_amd as plas
    text = open(os.path.join(ROOT, "include", "plas.h")).read()
    assert int(re.search(r"#define PLAS_ABI_VERSION (\d+)", text).group(1)) == plas.ABI_VERSION
