"""Writes gravity_wave_paper_curves.json: the simulated surface elevation of
the paper's gravity wave (Sec. 4.1), a*(t*) at x = 0, for each boundary
condition variant at L = 200, 400 and 800 cells, and the analytic model, as
printed in the paper's convergence figures of that section (one figure per
variant; the numbers are the plotted data series of the LaTeX source). Run
once, by hand, where the paper's source is available; the tests read only the
JSON."""
import json
import os
import re
import sys

SRC = sys.argv[1] if len(sys.argv) > 1 else "/root/reference/PAPER.md"
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "gravity_wave_paper_curves.json")


def series(lines):
    """(label, [(t, a)]) for every plotted table of one figure file."""
    out, cur, label = [], None, None
    for ln in lines:
        if ln.startswith("table {"):
            cur = []
            continue
        if cur is not None:
            if ln.startswith("}"):
                out.append([None, cur])
                cur = None
                continue
            t, a = ln.split()
            cur.append((float(t), float(a)))
            continue
        m = re.match(r"\\addlegendentry\{(.*)\}", ln)
        if m and out and out[-1][0] is None:
            out[-1][0] = m.group(1)
    return out


def main():
    text = open(SRC, encoding="utf-8").read().split("\n")
    files = {}
    name = None
    for ln in text:
        m = re.match(r"%% file: (\S+)", ln)
        if m:
            name = m.group(1)
            files[name] = []
            continue
        if name:
            files[name].append(ln.strip())
    res = {"source": "Sec. 4.1 (gravity wave), convergence figures of the four variants: surface "
                     "elevation a* at x = 0 over t* for L = 200, 400, 800, and the analytic model",
           "variants": {}, "model": None}
    for v in ("nbrc", "nbkc", "om", "om3"):
        for label, pts in series(files["figures/gravity-wave/convergence-%s.tex" % v]):
            m = re.search(r"L=(\d+)", label or "")
            if m:
                res["variants"].setdefault(v.upper(), {})[m.group(1)] = pts
            elif label and label.startswith("Analytical model") and res["model"] is None:
                res["model"] = pts
    with open(OUT, "w") as fh:
        json.dump(res, fh, separators=(",", ":"))
    print(OUT, {k: {L: len(p) for L, p in d.items()} for k, d in res["variants"].items()}, len(res["model"]))


if __name__ == "__main__":
    main()
