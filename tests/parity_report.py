"""Summarises the achieved parity margins that the GPU tests append to the
file named by PYRO_PARITY_LOG (one JSON object per line: case, quantity,
value, bar) as a markdown table, the worst value per (case, quantity).

    PYRO_PARITY_LOG=gpurun_out/parity.jsonl python -m pytest tests -m gpu -q
    python tests/parity_report.py gpurun_out/parity.jsonl > profiles/parity_margins.md
"""

import json
import sys


def main(path):
    worst = {}
    order = []
    for line in open(path):
        d = json.loads(line)
        key = (d["case"], d["quantity"])
        if key not in worst:
            order.append(key)
            worst[key] = d
        elif d["value"] > worst[key]["value"]:
            worst[key] = d
    print("# Achieved parity margins of the GPU tests\n")
    print("Worst value per test case and quantity over one run of the GPU suite on one")
    print("MI355X (errors against the CPU oracle unless the quantity says otherwise; the bar")
    print("is the test's assertion).  Produced by:\n")
    print("    PYRO_PARITY_LOG=gpurun_out/parity.jsonl python -m pytest tests -m gpu -q")
    print(f"    python tests/parity_report.py gpurun_out/parity.jsonl\n")
    print("| case | quantity | achieved | bar | bar / achieved |")
    print("|---|---|---|---|---|")
    for key in order:
        d = worst[key]
        v, b = d["value"], d["bar"]
        ratio = f"{b / v:.0f}" if v > 0 else "exact"
        print(f"| {d['case']} | {d['quantity']} | {v:.3e} | {b:.0e} | {ratio} |")


if __name__ == "__main__":
    main(sys.argv[1])
