"""Writes gamegen_sha256.json: the sha256 of the seeded input arrays of the
small configurations, so that any change to the generator's draws or
numbering is caught.  Run from the repository root:
    python tests/golden/make_gamegen_hashes.py
"""
import json
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
import gamegen as gg  # noqa: E402

out = {name: gg.make_config(name).sha256() for name in ("cfg1", "cfg2_d8")}
path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "gamegen_sha256.json")
with open(path, "w") as f:
    json.dump(out, f, indent=1, sort_keys=True)
    f.write("\n")
print(out)
