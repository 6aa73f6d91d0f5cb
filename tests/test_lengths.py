"""The library's length contract, on the host: every even length from 8 to
1024 that factors into 2, 3 and 5 has a transform schedule except the six
whose odd part no tile of the engine fits; nothing else has one."""
from paper_2202_14005_amd import _lib


def smooth235(n):
    for f in (2, 3, 5):
        while n % f == 0:
            n //= f
    return n == 1


UNSUPPORTED_SMOOTH = {450, 486, 750, 810, 900, 972}


def test_supported_lengths_are_exactly_the_contract():
    L = _lib.lib()
    for n in range(1, 1100):
        want = n % 2 == 0 and 8 <= n <= 1024 and smooth235(n) and n not in UNSUPPORTED_SMOOTH
        assert L.mrx_supported_length(n) == int(want), n
