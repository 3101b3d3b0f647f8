"""Write gg_ttggg_channel_tables.json: the oracle's tables for the gg -> t t~ g g g channel
weights, precomputed because the oracle takes about a minute for them.

  colour_weights  K_ds = sum over explicit colours |CF_ds|^2 of every amplitude entry
                  (Feynman diagram d, four-gluon colour structure s), in the order of
                  oracle.diagrams.entries("gg_ttggg"), with the entry's internal lines;
  good_helicities the helicity combinations the oracle's own filter keeps (1024 RAMBO events
                  of the fixed filter seed, max |M_h|^2 / |M|^2 > 1e-20).

Calls only oracle/ (test infrastructure); nothing comes from the HIP library.  Run from the
repository root:  python tests/golden/make_gg_ttggg_channel_tables.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import diagrams as Dg  # noqa: E402
from tests import workloads as W  # noqa: E402

NAME = "gg_ttggg"


def main():
    K = Dg.colour_weights_K(NAME)
    ents = Dg.entries(NAME)
    good = oracle.good_helicities(NAME, W.sqrt_s(NAME), W.final_masses(NAME), W.PARAMS)
    doc = {
        "process": NAME,
        "params": {"m_top": W.M_TOP, "alpha_em": W.ALPHA_EM, "alpha_s": W.ALPHA_S},
        "entries": [{"lines": list(Dg.descriptor(NAME, d)), "assign": list(s), "K": float(k)}
                    for (d, s), k in zip(ents, K)],
        "good_helicities": [int(h) for h in good],
    }
    with open(os.path.join(HERE, "gg_ttggg_channel_tables.json"), "w") as f:
        json.dump(doc, f, separators=(",", ":"))
        f.write("\n")


if __name__ == "__main__":
    main()
