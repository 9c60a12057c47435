"""Runs the oracle pins against one oracle library; exit 0 iff all pass.

Used by the mutation test: each planted mistake must make some pin fail.
"""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import oracle_pins  # noqa: E402

lib = sys.argv[1]
# optional: a name prefix of the pins to try first (the planted mistake's family)
first = sys.argv[2] if len(sys.argv) > 2 else ""
order = sorted(oracle_pins.PINS.items(), key=lambda kv: not (first and kv[0].startswith(first)))
for name, fn in order:
    try:
        fn(lib_path=lib)
    except AssertionError as e:
        print(f"caught by {name}: {e!r}"[:300])
        sys.exit(1)
try:
    oracle_pins.pin_ckdtree(lib_path=lib, n_tiles=16)
except AssertionError as e:
    print(f"caught by ckdtree: {e!r}"[:300])
    sys.exit(1)
print("not caught")
sys.exit(0)
