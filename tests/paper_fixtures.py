"""Readers of the text fixtures under tests/golden/ (values printed in the
paper, each file naming the passage it comes from)."""
import pathlib
from fractions import Fraction

import numpy as np

GOLDEN = pathlib.Path(__file__).parent / "golden"


def read_blocks(name: str) -> dict:
    """Parse a fixture.  '#' starts a comment; 'name = value' sets a scalar
    (kept as text); a line holding a single word opens a block, and every
    other line is a row (list of words) of the block opened last."""
    blocks, cur = {}, None
    for raw in (GOLDEN / name).read_text().splitlines():
        line = raw.split("#", 1)[0].strip()
        if not line:
            continue
        if "=" in line:
            key, value = (x.strip() for x in line.split("=", 1))
            blocks[key], cur = value, None
            continue
        tok = line.split()
        if len(tok) == 1:
            cur = blocks.setdefault(tok[0], [])
        elif cur is None:
            raise ValueError(f"{name}: row outside a block: {raw!r}")
        else:
            cur.append(tok)
    return blocks


def generator(blocks) -> np.ndarray:
    return np.array([[float(x) for x in r] for r in blocks["generator"]])


def embedded(blocks):
    return [[Fraction(x) for x in r] for r in blocks["embedded"]]


def same_digits(x: float, printed: str, decimals: int | None = None) -> bool:
    """True when x rounds to the printed value: to `decimals` decimals, else
    to as many significant digits as the printed mantissa shows."""
    v = float(printed)
    if decimals is None:
        mant = printed.lower().split("e")[0].lstrip("-")
        digits = len(mant.replace(".", "").lstrip("0"))
        decimals = digits - 1 - int(np.floor(np.log10(abs(v))))
    return abs(x - v) <= 0.5 * 10.0 ** -decimals * 1.001


def lognormal_params(blocks, s: int):
    """(mu, sigma) as s x s arrays from rows 'i-j mu sigma'; entries not
    listed get mu = 0, sigma = 1 (their embedded probability is zero)."""
    mu, sigma = np.zeros((s, s)), np.ones((s, s))
    for pair, m, sg in blocks["lognormal"]:
        i, j = (int(x) for x in pair.split("-"))
        mu[i, j], sigma[i, j] = float(m), float(sg)
    return mu, sigma


def embedded_matrix(blocks) -> np.ndarray:
    return np.array([[float(x) for x in r] for r in embedded(blocks)])
