"""ORACLE — test infrastructure only (only the test suite may import it).

Dictionary encoding of N-Triples text into integer triples (Section 6.2.1,
step 2): subjects and objects share one dictionary numbered from 0,
predicates have their own numbered from 1, each in order of first appearance
(reading the lines in order, a line's subject before its object). A term is
keyed by its text as written: an IRI with its angle brackets, a blank node
label with its "_:" prefix (ASCII letters, digits, "_" and "-"), a literal
with its quotes, escapes and any language tag (ASCII letters, digits and "-")
or datatype. Repeated lines stay repeated (a loader that takes the triples as
a set removes them). Written character by character; shares nothing with the
engine.
"""
from __future__ import annotations


class NTriplesError(ValueError):
    def __init__(self, line: int, msg: str):
        super().__init__(f"line {line}: {msg}")
        self.line = line


def _ascii_alnum(c: str) -> bool:
    return ("a" <= c <= "z") or ("A" <= c <= "Z") or ("0" <= c <= "9")


def _term(s: str, i: int, line: int):
    """The term starting at s[i] (no leading space): (text, next index)."""
    if s[i] == "<":
        j = s.find(">", i + 1)
        if j < 0:
            raise NTriplesError(line, "unterminated IRI")
        return s[i:j + 1], j + 1
    if s.startswith("_:", i):
        j = i + 2
        while j < len(s) and (_ascii_alnum(s[j]) or s[j] in "_-"):
            j += 1
        if j == i + 2:
            raise NTriplesError(line, "empty blank node label")
        return s[i:j], j
    if s[i] == '"':
        j = i + 1
        while True:
            if j >= len(s):
                raise NTriplesError(line, "unterminated literal")
            if s[j] == "\\":
                j += 2
                continue
            if s[j] == '"':
                break
            j += 1
        j += 1
        if j < len(s) and s[j] == "@":
            j += 1
            while j < len(s) and (_ascii_alnum(s[j]) or s[j] == "-"):
                j += 1
        elif s.startswith("^^<", j):
            k = s.find(">", j + 3)
            if k < 0:
                raise NTriplesError(line, "unterminated datatype IRI")
            j = k + 1
        return s[i:j], j
    raise NTriplesError(line, "a term starts with <, _: or a quote")


def encode(text: str):
    """(triples as a list of (s, p, o), vertex terms in id order, predicate terms in id
    order starting at id 1)."""
    vid, pid = {}, {}
    vertices, labels, triples = [], [], []
    for ln, raw in enumerate(text.split("\n"), start=1):
        s = raw.rstrip("\r")
        i = 0

        def skip(i):
            while i < len(s) and s[i] in " \t":
                i += 1
            return i

        i = skip(i)
        if i == len(s) or s[i] == "#":
            continue
        terms = []
        for _ in range(3):
            if i == len(s):
                raise NTriplesError(ln, "fewer than three terms")
            t, i = _term(s, i, ln)
            terms.append(t)
            i = skip(i)
        if i == len(s) or s[i] != ".":
            raise NTriplesError(ln, "a triple ends with '.'")
        i = skip(i + 1)
        if i < len(s) and s[i] != "#":
            raise NTriplesError(ln, "text after the final '.'")
        sub, pred, obj = terms
        if sub.startswith('"'):
            raise NTriplesError(ln, "a literal cannot be a subject")
        if not pred.startswith("<"):
            raise NTriplesError(ln, "a predicate is an IRI")
        ids = []
        for t in (sub, obj):
            if t not in vid:
                vid[t] = len(vertices)
                vertices.append(t)
            ids.append(vid[t])
        if pred not in pid:
            pid[pred] = len(labels) + 1
            labels.append(pred)
        triples.append((ids[0], pid[pred], ids[1]))
    return triples, vertices, labels
