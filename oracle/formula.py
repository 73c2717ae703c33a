"""Oracle for Kronecker-product formulas -- TEST INFRASTRUCTURE ONLY.

Only the test suite may import this module.  It shares no code with the GPU
library's formula front end: it has its own tokenizer and parser, and it
evaluates a formula from the definitions of its factors in fp64.

The language is the DSL of the paper's Section IV-A (Listing 1), with the
grammar of Listing 2: primaries DFT(n), I(n), twiddle(N, M), Permute(N, K)
and parenthesised expressions, joined by the Kronecker product and the
matrix product, both at one precedence level and grouping to the right.
Spellings: U+2297, "(x)" or "kron" for the Kronecker product; U+00B7, ".",
"*" or "@" for the matrix product; an identifier after a final matrix
product is the vector operand and is dropped.

Factors (Eq. 2 with the readings of its subscripts):
  DFT(n)        F[j, k] = w_n^(j k),  w_n = exp(-2 pi i / n)   (Section II)
  I(n)          identity
  twiddle(N, M) D^N_M: diagonal, entry i M + j = w_N^(i j), i < N/M, j < M
  Permute(N, K) Pi^N_K: (Pi x)[i M + j] = x[j K + i], M = N / K
The powers of w come from the C oracle's table (exact reduction of the
exponent mod n before the angle is formed).

Two evaluations:
  dense(text)          the formula's matrix: numpy kron and matmul of the
                       factor matrices (sizes up to a few thousand);
  apply(text, x)       F x row by row without forming F: a matrix product
                       applies right to left; A (x) B applies as
                       vec(A X B^T) on the row-major reshape X of x (the
                       Kronecker mixed-product identity); DFT(n) factors
                       use the O(n^2) C oracle.
"""
import re

import numpy as np

from . import dft as _oracle_dft
from . import twiddles as _oracle_twiddles

FORWARD = -1
INVERSE = +1
MAX_DIM = 1 << 24
_KEYWORDS = {"dft", "i", "identity", "twiddle", "permute"}

_TOKEN = re.compile(r"\s*(?:(?P<num>\d+)|(?P<name>[A-Za-z_][A-Za-z0-9_]*)|(?P<kron>⊗|\(x\))"
                    r"|(?P<mul>·|\.|\*|@)|(?P<punct>[(),]))")


def tokenize(text: str):
    out, pos = [], 0
    while pos < len(text):
        if text[pos:].strip() == "":
            break
        m = _TOKEN.match(text, pos)
        if not m:
            raise ValueError(f"unexpected character at offset {pos}: {text[pos]!r}")
        pos = m.end()
        kind = m.lastgroup
        val = m.group(kind)
        if kind == "name" and val.lower() == "kron":
            kind = "kron"
        out.append((kind, val))
    return out


class _Parser:
    def __init__(self, tokens):
        self.t = tokens
        self.i = 0

    def peek(self, k=0):
        return self.t[self.i + k] if self.i + k < len(self.t) else (None, None)

    def take(self, kind, val=None):
        tk = self.peek()
        if tk[0] != kind or (val is not None and tk[1] != val):
            raise ValueError(f"expected {val or kind} at token {self.i}, found {tk[1]!r}")
        self.i += 1
        return tk[1]

    def expr(self):
        # expr := primary [op expr]   (right grouping)
        left = self.primary()
        kind, _ = self.peek()
        if kind == "kron":
            self.i += 1
            return ("kron", left, self.expr())
        if kind == "mul":
            nxt = self.peek(1)
            if nxt[0] == "name" and nxt[1].lower() not in _KEYWORDS and self.i + 2 == len(self.t):
                self.i += 2  # trailing vector operand
                return left
            self.i += 1
            return ("mul", left, self.expr())
        return left

    def primary(self):
        kind, val = self.peek()
        if kind == "punct" and val == "(":
            self.i += 1
            e = self.expr()
            self.take("punct", ")")
            return e
        if kind != "name":
            raise ValueError(f"expected a factor at token {self.i}, found {val!r}")
        name = val.lower()
        self.i += 1
        self.take("punct", "(")
        a = int(self.take("num"))
        if name in ("dft", "i", "identity"):
            self.take("punct", ")")
            return ("dft" if name == "dft" else "id", a)
        if name in ("twiddle", "permute"):
            self.take("punct", ",")
            b = int(self.take("num"))
            self.take("punct", ")")
            return ("tw" if name == "twiddle" else "perm", a, b)
        raise ValueError(f"unknown factor {val!r}")


def parse(text: str):
    """Parse tree of nested tuples; raises ValueError on a syntax error."""
    p = _Parser(tokenize(text))
    tree = p.expr()
    if p.i != len(p.t):
        raise ValueError(f"unexpected token {p.peek()[1]!r} at token {p.i}")
    return tree


def size(tree) -> int:
    """Size under the shape rule; raises ValueError on a mismatch."""
    op = tree[0]
    if op in ("dft", "id"):
        if not 1 <= tree[1] <= MAX_DIM:
            raise ValueError(f"size {tree[1]} out of range")
        return tree[1]
    if op in ("tw", "perm"):
        n, m = tree[1], tree[2]
        if not (1 <= n <= MAX_DIM and m >= 1 and n % m == 0):
            raise ValueError(f"{op}({n}, {m}): second argument must divide the first")
        return n
    a, b = size(tree[1]), size(tree[2])
    if op == "kron":
        if a * b > MAX_DIM:
            raise ValueError("Kronecker product too large")
        return a * b
    if a != b:
        raise ValueError(f"matrix product of sizes {a} and {b}")
    return a


def _powers(n: int) -> np.ndarray:
    """w_n^t, t in [0, n), from the C oracle's table."""
    return _oracle_twiddles(n, FORWARD)


def dft_matrix(n: int) -> np.ndarray:
    j = np.arange(n)
    return _powers(n)[np.outer(j, j) % n]


def twiddle_diagonal(N: int, M: int) -> np.ndarray:
    """Entries of D^N_M: position i M + j holds w_N^(i j)."""
    t = np.arange(N)
    i, j = t // M, t % M
    return _powers(N)[(i * j) % N]


def permute_source(N: int, K: int) -> np.ndarray:
    """src[o] with (Pi^N_K x)[o] = x[src[o]]: o = i M + j reads j K + i."""
    M = N // K
    o = np.arange(N)
    i, j = o // M, o % M
    return j * K + i


def _dense(tree) -> np.ndarray:
    op = tree[0]
    if op == "dft":
        return dft_matrix(tree[1])
    if op == "id":
        return np.eye(tree[1], dtype=np.complex128)
    if op == "tw":
        return np.diag(twiddle_diagonal(tree[1], tree[2]))
    if op == "perm":
        N = tree[1]
        P = np.zeros((N, N), dtype=np.complex128)
        P[np.arange(N), permute_source(N, tree[2])] = 1
        return P
    A, B = _dense(tree[1]), _dense(tree[2])
    return np.kron(A, B) if op == "kron" else A @ B


def dense(text: str, sign: int = FORWARD) -> np.ndarray:
    """The formula's matrix (its complex conjugate for sign = +1)."""
    tree = parse(text)
    size(tree)
    F = _dense(tree)
    return F if sign == FORWARD else np.conj(F)


def _apply(tree, X: np.ndarray) -> np.ndarray:
    """F applied to each row of X (shape (rows, size(tree)))."""
    op = tree[0]
    if op == "dft":
        return _oracle_dft(X, FORWARD)
    if op == "id":
        return X
    if op == "tw":
        return X * twiddle_diagonal(tree[1], tree[2])[None, :]
    if op == "perm":
        return X[:, permute_source(tree[1], tree[2])]
    if op == "mul":
        return _apply(tree[1], _apply(tree[2], X))
    # Kronecker: (A (x) B) vec(Z) = vec(A Z B^T) with Z the (a, b) row-major view
    a, b = size(tree[1]), size(tree[2])
    rows = X.shape[0]
    Z = X.reshape(rows, a, b)
    Z = _apply(tree[2], Z.reshape(rows * a, b)).reshape(rows, a, b)           # Z B^T
    Z = np.ascontiguousarray(Z.transpose(0, 2, 1)).reshape(rows * b, a)
    Z = _apply(tree[1], Z).reshape(rows, b, a)                                  # A Z
    return np.ascontiguousarray(Z.transpose(0, 2, 1)).reshape(rows, a * b)


def apply(text: str, x, sign: int = FORWARD) -> np.ndarray:
    """F x for each row of x (1-D or 2-D), complex128; sign = +1 applies conj(F)."""
    tree = parse(text)
    n = size(tree)
    x = np.asarray(x)
    squeeze = x.ndim == 1
    X = np.ascontiguousarray(np.atleast_2d(x), dtype=np.complex128)
    if X.shape[1] != n:
        raise ValueError(f"rows of length {X.shape[1]} for a formula of size {n}")
    if sign == INVERSE:
        X = np.conj(X)
    Y = _apply(tree, X)
    if sign == INVERSE:
        Y = np.conj(Y)
    return Y[0] if squeeze else Y
