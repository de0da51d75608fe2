"""The committed counter summary that bench.py reads for roofline.traffic is
well formed: one fenced JSON block with the HBM bytes per launch of the tile
pass and of the Gram update, each with the source files its hash covers."""

import json
import re
from pathlib import Path

ROOT = Path(__file__).resolve().parents[1]


def test_traffic_block_parses():
    text = (ROOT / "profiles" / "traffic-haar64.md").read_text()
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    assert m, "no JSON block"
    rec = json.loads(m.group(1))
    N = 4096
    for kernel, floor in (("step", 4 * N * (N + 1)), ("gram", 2 * 4 * N * (N + 1))):
        r = rec[kernel]
        # at least the algorithmic bytes (H read once; the Gram also writes it)
        assert r["bytes_per_launch"] >= floor
        assert len(r["source_sha"]) == 16
        assert all((ROOT / f).exists() for f in r["files"])
