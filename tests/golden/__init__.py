"""Readers for the fixtures in this folder: numbers the paper prints, transcribed
by hand with their citation in each file's header.  The one computed fixture,
scf_si35_oracle.json, is written by make_scf_si35.py from the oracle alone."""
from __future__ import annotations

from pathlib import Path
from typing import NamedTuple

HERE = Path(__file__).resolve().parent


class TableIRow(NamedTuple):
    name: str
    n_si: int
    n_h: int
    h_bohr: float
    diameter_nm: float
    grid_points: int
    states: int
    scf_steps: int


def _rows(name):
    for line in (HERE / name).read_text().splitlines():
        line = line.strip()
        if line and not line.startswith("#"):
            yield line.split()


def table_i() -> list[TableIRow]:
    out = []
    for f in _rows("table_i.txt"):
        out.append(TableIRow(f[0], int(f[1]), int(f[2]), float(f[3]), float(f[4]),
                             int(f[5]), int(f[6]), int(f[7])))
    return out


def text_figures() -> dict[str, float]:
    return {f[0]: float(f[1]) for f in _rows("text_figures.txt")}
