"""Readers for the text fixtures under tests/golden/."""
import json
import os
from typing import List

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_paths(name: str) -> List[List[int]]:
    out = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                out.append([int(x) for x in line.split()])
    return out


def workloads() -> dict:
    with open(os.path.join(GOLDEN, "workloads.json")) as f:
        return json.load(f)


def read_labelled_paths(name: str) -> dict:
    """{label: [path, ...]} from lines "label: v v v" ('#' comments)."""
    out: dict = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split(":", 1)
                out.setdefault(k.strip(), []).append([int(x) for x in v.split()])
    return out
