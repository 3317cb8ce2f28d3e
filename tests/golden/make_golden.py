"""Writes the stored expected values under tests/golden/ (calls only oracle/).

    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from paper_2309_16724_amd.synth.integrals import make_integrals  # noqa: E402
from oracle.fock import fci  # noqa: E402


def main():
    h, eri = make_integrals(8, 0)
    e0 = fci(h, eri, 8, 0)[0]
    e1 = fci(h, eri, 8, 2)[0]
    out = {"system": "L=8 orbitals, N=8, integral seed 0",
           "source": "oracle.fock.fci (dense diagonalisation, 4900 determinants for M_S=0)",
           "E_fci_S0": float(e0), "E_fci_S1": float(e1)}
    with open(os.path.join(HERE, "fci_L8_seed0.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(out)


if __name__ == "__main__":
    main()
