"""The half-width LDS exchange's addressing (stockham_half.h), checked on the
CPU for every compiled list it can run: the kernel addresses each element it
writes as one per-butterfly base plus a compile-time offset,
  lds_pad(base + r NS) = lds_pad(base) + r NS + floor(r NS / 16),
and each element it reads as lds_pad(t) + (i TPT + r N/R) 17 / 16.  Both
identities must hold for every thread, butterfly and r, or elements land in
the wrong LDS word.  A replay of the whole exchange sequence in NumPy then
checks that the stages, addressed this way, compute the DFT."""
import numpy as np
import pytest

from paper_2207_06803_amd import fftc

LDS_MAX = 163840


def lds_pad(x):
    return x + (x >> 4)


def half_lists():
    """(dtype bytes, N, radices, TPT) for the compiled lists the half-width
    exchange can take: power-of-two radices, a full exchange over a quarter
    of the LDS, and a thread count that gives every stage N / TPT elements
    per thread."""
    out = []
    for dtype, cs in (("c64", 8), ("c128", 16)):
        for n, rs in fftc.compiled_lists(dtype):
            if len(rs) < 2 or any(r & (r - 1) for r in rs):
                continue
            if lds_pad(n) * cs <= LDS_MAX // 4:
                continue
            for tpt in (64, 128, 256, 512, 1024):
                if all((n // r) % tpt == 0 for r in rs) and tpt % 16 == 0:
                    out.append((cs, n, tuple(rs), tpt))
    return out


CASES = half_lists()


def test_there_are_lists_to_check():
    ns = {(cs, n) for cs, n, _, _ in CASES}
    assert (8, 16384) in ns and (8, 8192) in ns and (16, 8192) in ns and (16, 4096) in ns
    assert (8, 32768) in ns and (16, 16384) in ns  # the wide lengths


@pytest.mark.parametrize("cs,n,rs,tpt", CASES)
def test_write_and_read_offsets(cs, n, rs, tpt):
    t = np.arange(tpt)[:, None, None]
    ns = 1
    for q, r in enumerate(rs):
        nr = n // r
        nb = nr // tpt
        i = np.arange(nb)[None, :, None]
        k = np.arange(r)[None, None, :]
        j = t + i * tpt
        base = (j // ns) * ns * r + j % ns
        assert np.array_equal(lds_pad(base) + k * ns + (k * ns) // 16, lds_pad(base + k * ns))
        if q + 1 < len(rs):
            r2 = rs[q + 1]
            nr2 = n // r2
            i2 = np.arange(nr2 // tpt)[None, :, None]
            k2 = np.arange(r2)[None, None, :]
            assert np.array_equal(lds_pad(t) + (i2 * tpt + k2 * nr2) // 16 * 17,
                                  lds_pad(t + i2 * tpt + k2 * nr2))
        ns *= r


def test_exchange_sequence_computes_the_dft():
    """Replay of the kernel's stages for one 4096-point list with its
    addressing (real and imaginary parts through the same array) against
    numpy.fft."""
    n, rs, tpt = 4096, (16, 16, 16), 256
    x = np.random.default_rng(5).standard_normal(n) + 1j * np.random.default_rng(6).standard_normal(n)
    e = n // tpt
    t = np.arange(tpt)
    r1 = rs[0]
    v = np.stack([x[t + i * tpt + k * (n // r1)] for i in range(e // r1) for k in range(r1)], axis=1)
    ns = 1
    lds = np.full(lds_pad(n), np.nan)
    for q, r in enumerate(rs):
        nr = n // r
        nb = nr // tpt
        out = np.empty_like(v)
        for i in range(nb):
            j = t + i * tpt
            blk = v[:, i * r:(i + 1) * r]
            if ns > 1:
                blk = blk * np.exp(-2j * np.pi * np.outer(j % ns, np.arange(r)) / (ns * r))
            out[:, i * r:(i + 1) * r] = np.fft.fft(blk, axis=1)
        addrs = np.stack([lds_pad((t + i * tpt) // ns * ns * r + (t + i * tpt) % ns) + k * ns + (k * ns) // 16
                          for i in range(nb) for k in range(r)], axis=1)
        if q + 1 == len(rs):
            y = np.empty(n, complex)
            lds[:] = np.nan
            lds[addrs] = out.real
            re = lds[lds_pad(np.arange(n))]
            lds[addrs] = out.imag
            y = re + 1j * lds[lds_pad(np.arange(n))]
            break
        r2 = rs[q + 1]
        nr2 = n // r2
        raddr = np.stack([lds_pad(t) + (i * tpt + k * nr2) // 16 * 17 for i in range(nr2 // tpt) for k in range(r2)],
                         axis=1)
        lds[:] = np.nan
        lds[addrs] = out.real
        vr = lds[raddr]
        lds[addrs] = out.imag
        v = vr + 1j * lds[raddr]
        ns *= r
    assert np.allclose(y, np.fft.fft(x), rtol=0, atol=1e-9 * np.abs(np.fft.fft(x)).max())
