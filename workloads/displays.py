"""Lenticular display parameters (paper section 3.1).

A display is described by its panel size W x H (pixels; three RGB subpixels
per pixel), the number of views N, and the three lens parameters of the
view-index map: slant tan(alpha), grating pitch L_x (in subpixels) and the
lens-to-panel offset K_offset.  The lens parameters are kept as exact
rationals so that the integer view-index map is reproducible bit for bit.
"""
from __future__ import annotations

import dataclasses
from fractions import Fraction


@dataclasses.dataclass(frozen=True)
class Rational:
    num: int
    den: int = 1

    def __post_init__(self):
        if self.den <= 0:
            raise ValueError("denominator must be positive")

    @staticmethod
    def of(x) -> "Rational":
        if isinstance(x, Rational):
            return x
        f = Fraction(x).limit_denominator(10 ** 9)
        return Rational(f.numerator, f.denominator)

    def fraction(self) -> Fraction:
        return Fraction(self.num, self.den)

    def __float__(self):
        return self.num / self.den


@dataclasses.dataclass(frozen=True)
class DisplayParams:
    width: int
    height: int
    num_views: int
    tan_slant: Rational
    pitch: Rational
    offset: Rational = Rational(0, 1)
    tile_w: int = 16
    tile_h: int = 16

    def with_tile(self, tw: int, th: int) -> "DisplayParams":
        return dataclasses.replace(self, tile_w=tw, tile_h=th)

    @property
    def num_subpixels(self) -> int:
        return 3 * self.width * self.height
