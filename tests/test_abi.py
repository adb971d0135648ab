"""The C ABI library: builds, loads and exports every symbol include/chem.h declares (no GPU)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "chem.h")).read()
    return sorted(set(re.findall(r"\b(chem_[a-z_A-Z0-9]+)\s*\(", text)))


def test_header_and_binding_agree():
    from paper_2510_10005_amd._binding import EXPORTED
    assert sorted(EXPORTED) == _declared()


def test_library_exports_every_declared_symbol():
    lib_path = os.path.join(ROOT, "paper_2510_10005_amd", "libchem.so")
    if not os.path.exists(lib_path):
        pytest.skip("libchem.so not built")
    lib = ctypes.CDLL(lib_path)
    for name in _declared():
        assert hasattr(lib, name), name


def test_host_side_calls_without_gpu():
    from paper_2510_10005_amd import _binding as b
    lib = b.load()
    o = b.default_options()
    assert o.method == 0 and o.newton_max == 10 and o.halving_max_depth == 8 and o.rtol == 1e-6
    assert lib.chem_error_string(3) == b"mechanism parse error"
    h = ctypes.c_void_p()
    assert lib.chem_load_mechanism(b"/nonexistent.json", None, ctypes.byref(h)) == 3
    assert b"cannot read" in lib.chem_last_error_message()


def test_precompile_generated_kernels(tmp_path):
    from paper_2510_10005_amd import _binding as b
    from synth import mechanism_file
    path = b.precompile(mechanism_file("tiny_5_6"), str(tmp_path))
    assert os.path.getsize(path) > 1000
    bad = tmp_path / "bad.json"
    bad.write_text('{"species": [], "reactions": []}')
    with pytest.raises(b.ChemError) as e:
        b.precompile(str(bad), str(tmp_path))
    assert e.value.code == 3


def test_options_struct_layout_matches_header(tmp_path):
    """The ctypes mirror of chem_integrator_opts has the C compiler's offsets and size."""
    from paper_2510_10005_amd._binding import IntegratorOptions
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    fields = [f for f, _ in IntegratorOptions._fields_]
    src = tmp_path / "layout.c"
    body = "\n".join(f'  printf("{f} %zu\\n", offsetof(chem_integrator_opts, {f}));' for f in fields)
    src.write_text("#include <stddef.h>\n#include <stdio.h>\n#include \"chem.h\"\nint main(void) {\n" + body +
                   '\n  printf("sizeof %zu\\n", sizeof(chem_integrator_opts));\n  return 0;\n}\n')
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                       check=True).stdout.splitlines())
    for f in fields:
        assert int(out[f]) == getattr(IntegratorOptions, f).offset, f
    assert int(out["sizeof"]) == ctypes.sizeof(IntegratorOptions)
    from paper_2510_10005_amd import _binding as b
    if os.path.exists(os.path.join(ROOT, "paper_2510_10005_amd", "libchem.so")):
        o = b.default_options()
        assert o.probe_attempts == 48 and o.reserved_ == 0


def test_mechanism_above_block_limit_is_rejected(tmp_path):
    """States of more than 160 components are refused at parse time (no code is generated): the
    150-species mechanism with ten more (inert, copied) species."""
    import json
    from paper_2510_10005_amd import _binding as b
    from synth import mechanism_file
    lib = b.load()
    m = json.load(open(mechanism_file("large_150_1000")))
    extra = []
    for k in range(10):
        sp = dict(m["species"][-1])
        sp["name"] = f"XTRA{k}"
        extra.append(sp)
    m["species"] += extra
    path = tmp_path / "too_large.json"
    path.write_text(json.dumps(m))
    buf = ctypes.create_string_buffer(4096)
    assert lib.chem_precompile(str(path).encode(), None, buf, 4096) == 7       # CHEM_EUNSUPPORTED
    assert b"at most 159 are supported" in lib.chem_last_error_message()
