"""Host logic of bench.py (no GPU): the roofline's counted HBM traffic is
reported only while the kernel source, its launch constants and the table's
rows per block are the ones the committed counter summary was taken on."""
import hashlib

import bench


def _tree(tmp_path, kernel=b"kernel source", header="constexpr int kSpecCap = 262144;\n#define MSV_LU_GROUPS 2\n"):
    csrc = tmp_path / "paper_1810_07067_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "tabulate.hip").write_bytes(kernel)
    (csrc / "msv_internal.h").write_text(header)
    (tmp_path / "profiles").mkdir()
    return hashlib.sha256(kernel).hexdigest()


def _profile(tmp_path, text):
    (tmp_path / "profiles" / "t.md").write_text(text)


def test_counted_bytes_follow_source_constants_and_rows(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h = _tree(tmp_path)
    good = f"    tabulate.hip sha256 = {h}\n    kSpecCap = 262144\n    rows per block = 128\n    tab bytes = 1234\n"
    _profile(tmp_path, good)
    get = lambda rows=128, consts=("kSpecCap",): bench._counted_bytes("t.md", "tabulate.hip", consts, "tab bytes",
                                                                        rows=rows)
    assert get() == 1234
    assert get(rows=None) == 1234        # rows not part of this gate
    assert get(rows=512) is None          # counted on other row blocks
    assert get(consts=("kSpecCap", "MSV_LU_GROUPS")) is None  # a constant the summary does not record
    _profile(tmp_path, good.replace("kSpecCap = 262144", "kSpecCap = 65536"))
    assert get() is None                  # counted with another launch constant
    _profile(tmp_path, good.replace(h, "0" * 64))
    assert get() is None                  # counted on another source
    _profile(tmp_path, good)
    (tmp_path / "paper_1810_07067_amd" / "csrc" / "tabulate.hip").write_bytes(b"kernel source, edited")
    assert get() is None                  # the source changed since


def test_internal_constant_reads_constexpr_and_macro_defaults(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    _tree(tmp_path)
    assert bench._internal_constant("kSpecCap") == "262144"
    assert bench._internal_constant("MSV_LU_GROUPS") == "2"
    assert bench._internal_constant("kMissing") is None
