"""The two-pass plans' pass-1 factors D^N_M (Eq. 2), as the compiled column
kernels form them (fourstep_spec.h), replayed in integer exponents on the CPU:
a thread stores rows p of columns c = c0 + s S of its tile, loads
w_N^{(col0 + c0) p} and the powers w_N^{2^b S p} (b < log2 of the stores per
row, from the table of w_N^{c p}, c below the tile width), and forms the
factor of store s as the factor of store s - 2^b (b = the top bit of s) times
one loaded power.  Every store must end with exponent (col0 + c) p, and every
loaded power must come from a row of that table (2^b S below the tile
width)."""
import pytest


def ilog2_ceil(x):
    return 0 if x <= 1 else 1 + ilog2_ceil((x + 1) // 2)


# (column length LEN, threads per column TPT, columns per tile TC): the
# shapes of the compiled column kernels (16 complex64 or 8 complex128 columns,
# TPT from the Stockham lists of lengths 2..1024), including ones whose
# threads cover several rows (LEN > NTH) and several columns (NTH > LEN)
SHAPES = [(16, 1, 16), (64, 4, 16), (128, 8, 16), (256, 16, 16), (512, 64, 16), (1024, 64, 16),
          (256, 16, 8), (1024, 64, 8), (96, 8, 16), (48, 4, 16), (320, 32, 16), (32, 2, 16), (8, 1, 8)]


@pytest.mark.parametrize("LEN,TPT,TC", SHAPES)
def test_pass1_factor_chain(LEN, TPT, TC):
    NTH = TPT * TC
    TOT = TC * LEN
    IT = -(-TOT // NTH)
    if not (NTH % LEN == 0 or LEN % NTH == 0):
        pytest.skip("rows do not repeat per thread: the kernel reads both tables per element")
    PP = 1 if NTH % LEN == 0 else LEN // NTH
    S = NTH // LEN if NTH % LEN == 0 else 1
    CN = -(-IT // PP)
    NB = ilog2_ceil(CN)
    for col0 in (0, TC, 5 * TC):
        for tid in range(NTH):
            c0 = tid // LEN if NTH % LEN == 0 else 0
            a = [(col0 + c0) * ((tid % LEN) + pp * NTH) for pp in range(PP)]   # exponents
            pw = [[((S << b) % TC) * ((tid % LEN) + pp * NTH) for b in range(NB)] for pp in range(PP)]
            for pp in range(PP):
                for b in range(NB):
                    assert (S << b) < TC  # a real row of the table, the modulo never wraps
            v = [None] * IT
            for i in range(IT):
                l = tid + i * NTH
                c, p = l // LEN, l % LEN
                pp, s = i % PP, i // PP
                if s == 0:
                    v[i] = a[pp]
                else:
                    hb = s.bit_length() - 1
                    v[i] = v[i - (PP << hb)] + pw[pp][hb]
                if l < TOT:
                    assert p == (tid % LEN) + pp * NTH
                    assert v[i] == (col0 + c) * p, (tid, i, c, p)
