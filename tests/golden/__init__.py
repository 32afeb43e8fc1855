"""Values printed in the paper, read from paper_values.txt (each line cites
the passage it comes from)."""
import os


def paper_values():
    out = {}
    path = os.path.join(os.path.dirname(__file__), "paper_values.txt")
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            k, v = (t.strip() for t in line.split("=", 1))
            out[k] = float(v) if "." in v else int(v)
    return out
