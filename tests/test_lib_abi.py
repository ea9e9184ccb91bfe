"""The C-ABI library builds, loads, and exports every symbol include/amm.h
declares (no compute call: there may be no GPU)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, 'paper_1909_08015_amd', 'libamm.so')


def declared_symbols():
    src = open(os.path.join(ROOT, 'include', 'amm.h')).read()
    src = re.sub(r'/\*.*?\*/', '', src, flags=re.S)
    return sorted(set(re.findall(r'\b(amm_[a-z_0-9]+)\s*\(', src)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ('amm_create', 'amm_enumerate', 'amm_build_tables', 'amm_integrate', 'amm_read',
              'amm_sample', 'amm_eval', 'amm_profile', 'amm_mlp_train'):
        assert s in syms


@pytest.mark.skipif(not os.path.exists(LIB), reason='libamm.so not built')
def test_library_exports_every_declared_symbol():
    out = subprocess.run(['nm', '-D', '--defined-only', LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r' T (amm_[a-z_0-9]+)', out))
    missing = [s for s in declared_symbols() if s not in exported]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason='libamm.so not built')
def test_binding_loads_and_reports_errors_without_gpu():
    from paper_1909_08015_amd import amm
    L = amm.lib()
    for name in amm.SYMBOLS:
        assert hasattr(L, name)
    # an argument error is reported through amm_last_error, no crash
    assert L.amm_enumerate(None, 3, None, None, None) == -1
    assert b'ctx' in L.amm_last_error()


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_1909_08015_amd import amm
    monkeypatch.setattr(amm, 'LIB_PATH', str(tmp_path / 'nope.so'))
    monkeypatch.setattr(amm, '_lib', None)
    with pytest.raises(amm.AmmError):
        amm.lib()
