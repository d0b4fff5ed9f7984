"""The paper's printed numbers (tests/golden/paper_values.json, each entry with
the passage it comes from)."""
import json
import os

_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_values.json")
_DATA = None


def paper(key):
    """The entry ``key``: a dict with at least "value" and "source"."""
    global _DATA
    if _DATA is None:
        with open(_PATH) as f:
            _DATA = json.load(f)
    return _DATA[key]
