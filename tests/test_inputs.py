"""The seeded synthetic workloads regenerate exactly: pair count, base
count and SHA-256 of every workload at seed 0 match the committed manifest
(tests/golden/seqgen_manifest.txt, written by make_manifest.py beside it)."""

import os

import pytest

import seqgen

MANIFEST = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "seqgen_manifest.txt")


def _entries():
    rows = []
    for line in open(MANIFEST):
        if line.strip() and not line.startswith("#"):
            name, n, bases, digest = line.split()
            rows.append((name, int(n), int(bases), digest))
    return rows


@pytest.mark.parametrize("workload,n_pairs,bases,digest", _entries())
def test_workload_matches_manifest(workload, n_pairs, bases, digest):
    b = seqgen.make_workload(workload)
    assert b.n_pairs == n_pairs
    assert int(b.t_len.sum() + b.q_len.sum()) == bases
    assert b.digest() == digest
