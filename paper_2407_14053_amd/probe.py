"""Print the device's measured vector-ALU issue rates (``dl_probe_issue_rates``) as one JSON line, with the
per-compute-unit, per-clock figures they imply.  Usage: ``python -m paper_2407_14053_amd.probe [device]``."""
import json
import sys

from paper_2407_14053_amd import api


def main():
    dev = int(sys.argv[1]) if len(sys.argv) > 1 else 0
    r = api.probe_issue_rates(dev)
    cu, hz = r["compute_units"], r["engine_clock_hz"]
    per = {k.replace("_per_s", "_per_cu_clock"): v / (cu * hz) for k, v in r.items() if k.endswith("_per_s")} \
        if hz > 0 else {}
    print(json.dumps({**r, **per}), flush=True)


if __name__ == "__main__":
    main()
