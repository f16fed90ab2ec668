"""Host FASTA ingest (hmsv_fasta_parse): a fixture of made-up sequences
covering line wraps, lower case, stop and gap symbols, digits, an empty
record, CRLF line ends and degenerate letters, checked against a plain
parse written here; a round trip of synthetic sequences; and errors."""
import os

import numpy as np
import pytest

import synth

hm = pytest.importorskip("paper_1707_09683_amd")

FIXTURE = os.path.join(os.path.dirname(__file__), "golden", "synthetic.fasta")
CODE = {c: i for i, c in enumerate(synth.ALPHABET)}
CODE.update({"B": 21, "J": 22, "Z": 23, "U": 24, "O": 25, "X": 26})


def plain_parse(text):
    heads, seqs = [], []
    for line in text.split("\n"):
        line = line.rstrip("\r")
        if line.startswith(">"):
            heads.append(line[1:])
            seqs.append([])
        else:
            for ch in line.upper():
                if ch in CODE:
                    seqs[-1].append(CODE[ch])
    return heads, seqs


def test_fixture_matches_plain_parse():
    text = open(FIXTURE, "rb").read()
    heads, res, off = hm.parse_fasta(text)
    eh, es = plain_parse(text.decode())
    assert heads == eh and len(heads) == 5
    assert [list(res[off[i]:off[i + 1]]) for i in range(len(heads))] == es
    # by hand: lengths 22, 13, 0, 20, 8; syn2 is M K V B J Z U O X A G G R
    assert list(np.diff(off)) == [22, 13, 0, 20, 8]
    assert list(res[off[1]:off[2]]) == [10, 8, 17, 21, 22, 23, 24, 25, 26, 0, 5, 5, 14]
    assert heads[4] == "syn5 CRLF line ends"


def test_round_trip_of_synthetic_sequences():
    rng = np.random.default_rng(3)
    L = rng.integers(0, 300, size=200).astype(np.int64)
    res, off = synth.sample_residues(rng, L)
    res[rng.random(res.size) < 0.02] = 26
    letters = np.array(list(synth.ALPHABET) + ["?"] + list("BJZUOX"))
    out = []
    for i in range(len(L)):
        s = "".join(letters[res[off[i]:off[i + 1]]])
        out.append(f">s{i}\n" + "\n".join(s[k:k + 60] for k in range(0, len(s), 60)))
    heads, r2, o2 = hm.parse_fasta("\n".join(out) + "\n")
    assert heads == [f"s{i}" for i in range(len(L))]
    assert np.array_equal(o2, off) and np.array_equal(r2, res)


def test_errors_and_empty_input():
    assert hm.parse_fasta(b"")[0] == []
    with pytest.raises(hm.HmsvError, match="byte 0"):
        hm.parse_fasta(b"ACDE\n>x\nAC\n")            # residues before any header
    with pytest.raises(hm.HmsvError, match="byte 5"):
        hm.parse_fasta(b">x\nAC#D\n")                # not a residue letter
