"""Error statements of the GPU parity cases.

Every parity case reports, next to its pass/fail bar, the error it measured
against the FP64 oracle:
  rel_l2  = |got - ref|_2 / |ref|_2 over the compared elements;
  max_rel = max_i |got_i - ref_i| / max(|ref_i|, 1e-3 max_j |ref_j|)
            (elements far below the largest are measured against that floor).
Each case prints one "[parity]" line; with SM_PARITY_LOG set, it is also
appended to that file as JSON.  Run as a script, this module turns such a
log into the text table kept under profiles/:
    python tests/_errlog.py LOG.jsonl OUT.txt "command that produced the log"
"""
import json
import os
import sys

import numpy as np


def errors(got, ref):
    got = np.asarray(got, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    if ref.size == 0:
        return 0.0, 0.0
    diff = got - ref
    rel = float(np.linalg.norm(diff) / max(float(np.linalg.norm(ref)), 1e-300))
    floor = max(1e-3 * float(np.abs(ref).max()), 1e-300)
    mx = float((np.abs(diff) / np.maximum(np.abs(ref), floor)).max())
    return rel, mx


def record(case, got, ref, bar):
    """Log the errors of one comparison; returns (rel_l2, max_rel)."""
    rel, mx = errors(got, ref)
    note(case, rel, mx, int(np.size(ref)), bar)
    return rel, mx


def note(case, rel, mx, n, bar, kind="rel_l2"):
    """Log an error computed by the caller (kind names what `rel` is)."""
    print("[parity] %-58s %s=%.3e max_rel=%.3e n=%d bar=%.0e" % (case, kind, rel, mx, n, bar), flush=True)
    path = os.environ.get("SM_PARITY_LOG")
    if path:
        with open(path, "a") as fh:
            fh.write(json.dumps({"case": case, "kind": kind, "err": rel, "max_rel": mx, "n": n,
                                 "bar": bar}) + "\n")


def digest(log, out, command):
    rows = [json.loads(l) for l in open(log) if l.strip()]
    lines = ["# Measured errors of the GPU parity cases against the FP64 oracle",
             "command: %s" % command,
             "err: relative L2 (kind rel_l2), or the normalised mismatch the case states (kind)",
             "max_rel: max |got - ref| / max(|ref|, 1e-3 max|ref|) over the compared elements",
             "", "%-72s %-11s %10s %10s %10s %8s" % ("case", "kind", "err", "max_rel", "n", "bar")]
    for r in rows:
        lines.append("%-72s %-11s %10.3e %10.3e %10d %8.0e" % (r["case"][:72], r["kind"], r["err"],
                                                             r["max_rel"], r["n"], r["bar"]))
    worst = {}
    for r in rows:
        key = "fp64" if "fp64" in r["case"] else "fp32"
        if r["kind"] == "rel_l2":
            worst[key] = max(worst.get(key, 0.0), r["err"] / r["bar"])
    lines += ["", "cases: %d; largest err / bar: %s" % (len(rows), ", ".join(
        "%s %.2e" % kv for kv in sorted(worst.items())))]
    text = "\n".join(lines) + "\n"
    with open(out, "w") as fh:
        fh.write(text)
    print(text, end="")


if __name__ == "__main__":
    digest(sys.argv[1], sys.argv[2], sys.argv[3] if len(sys.argv) > 3 else "")
