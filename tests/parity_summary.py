"""Summary of the per-point parity records a GPU test session writes to
parity/records.jsonl under the results folder (helpers.record): per test, the points and
output kinds compared, the largest error, the bars used, and whether every bar
was the plain one.

    python tests/parity_summary.py <results folder>/parity/records.jsonl > profiles/parity_bars.md
"""
import collections
import json
import sys


def main(path):
    rows = [json.loads(line) for line in open(path)]
    by = collections.OrderedDict()
    for r in rows:
        by.setdefault(r["test"], []).append(r)
    print("Parity of the GPU path against the oracle, from the records of one session of "
          "`python -u -m pytest tests -m gpu -x -v --timeout 300 --timeout-method thread`, summarised by "
          f"`python tests/parity_summary.py {path} > profiles/parity_bars.md`.")
    print()
    print("| test | comparisons | points | max error | bars used | max oracle spread | max conditioning proxy |")
    print("|---|---|---|---|---|---|---|")
    plain_tests = []
    for t, rs in by.items():
        bars = sorted({r["bar"] for r in rs})
        spreads = [r["spread"] for r in rs if r["spread"] is not None]
        kap = [r["kappa"] for r in rs if r["kappa"] is not None]
        pts = len({(r["E"], r.get("side"), r.get("b"), r.get("point")) for r in rs})
        chosen = "fp32" in t or "refine" in t
        barcol = ("1e-10 (plain)" if bars == [1e-10] else
                  "1e-6 (chosen form)" if bars == [1e-6] and chosen else
                  f"{bars[0]:.1e}" if len(bars) == 1 else f"{min(bars):.1e} .. {max(bars):.1e}")
        if bars == [1e-10]:
            plain_tests.append(t)
        print(f"| {t} | {len(rs)} | {pts} | {max(r['err'] for r in rs):.2e} | {barcol} | "
              f"{max(spreads) if spreads else float('nan'):.1e} | {max(kap) if kap else float('nan'):.1e} |")
    worst = max((r for r in rows if r["test"] in plain_tests), key=lambda r: r["err"], default=None)
    print()
    print(f"{len(rows)} comparisons in {len(by)} tests; {len(plain_tests)} tests held every comparison to the plain "
          f"1e-10 bar" + (f" (largest error there {worst['err']:.2e}, {worst['test']}, E = {worst['E']:+.4f}, "
                          f"{worst['name']})." if worst else "."))


if __name__ == "__main__":
    main(sys.argv[1])
