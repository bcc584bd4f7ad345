"""Values the paper prints (setups and results of its Section 5 tests),
kept as cited text fixtures under tests/golden/."""
import json
import os

_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name: str) -> dict:
    with open(os.path.join(_DIR, name)) as f:
        return json.load(f)
