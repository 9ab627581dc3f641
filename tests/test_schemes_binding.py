"""Host-side scheme names of the binding match the header's enum (no GPU needed)."""
import re
from pathlib import Path

from paper_0910_0992_amd import _lib as L
from oracle.schemes import SCHEMES

HEADER = Path(__file__).resolve().parent.parent / "include" / "tprec.h"


def test_scheme_enum_matches_header():
    text = HEADER.read_text()
    enum = {m.group(1): int(m.group(2)) for m in re.finditer(r"\bTP_([A-Z0-9_]+)\s*=\s*(\d+)", text)}
    for name, value in L.SCHEMES.items():
        assert enum[name] == value, name


def test_binding_knows_every_oracle_scheme():
    assert set(SCHEMES) == set(L.SCHEMES)
