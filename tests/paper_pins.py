"""Shared helpers for the oracle pins: paper values and CGS constants."""
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def paper_values():
    with open(os.path.join(HERE, "golden", "paper_values.json")) as f:
        return json.load(f)


def cgs():
    c = paper_values()["constants_cgs"]
    out = dict(k_B=c["k_B"], m_p=c["m_p"], c=c["c"])
    out["a_r"] = 4.0 * c["sigma_SB"] / c["c"]  # a_r = 4 sigma / c (Sect. 2)
    return out
