"""Writes the decay values of taylor_green_decay.json from the printed formula.

Uses only the exact Taylor-Green solution (section 4.1, eq. tgv); no code of
the oracle or of the HIP path is involved.
"""
import json
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    path = os.path.join(HERE, "taylor_green_decay.json")
    with open(path) as f:
        doc = json.load(f)
    for c in doc["cases"]:
        c["decay"] = math.exp(-8.0 * math.pi ** 2 / c["re"] * c["t"])
    with open(path, "w") as f:
        json.dump(doc, f, indent=2)
        f.write("\n")


if __name__ == "__main__":
    main()
