"""Reader of tests/golden/paper_claims.txt: numbers the paper states, each with its
citation in the file, as a dict name -> float."""
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_claims.txt")


def paper_claims():
    out = {}
    for line in open(GOLDEN):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        k, v = (x.strip() for x in line.split("="))
        out[k] = float(v)
    return out
