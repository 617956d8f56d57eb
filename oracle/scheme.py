"""Pipeline configuration and retrieval targets (oracle side).

The configuration space follows Table I (tuning configurations): interpolation
scheme (per-level, or per-region with one of the d! dimension orders),
coefficient decomposition along one of d directions or none, and the encoding
(generic bitplane, or negabinary digit planes with or without XOR chaining),
optionally followed by the lossless stage on the stored planes
(``oracle.bitplane``).  Interpolation degree 3 is the
paper's cubic choice (Section IV); degree 1 is the multilinear form the paper
starts from.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional, Tuple


@dataclass(frozen=True)
class Scheme:
    kind: str = "level"              # "level" (per-level) or "region" (per-region)
    degree: int = 3                  # 1 = linear, 3 = cubic
    order: Optional[Tuple[int, ...]] = None   # per-region pass order (axes); None = fastest first
    cd_axis: Optional[int] = None    # stacking axis of coefficient decomposition; None = off
    levels: Optional[int] = None     # number of levels L; None = default
    lossless: bool = False           # zero-word suppression of the magnitude planes
    encoding: str = "generic"        # "generic", "negabinary" or "negabinary_xor" (Table I)

    def pass_order(self, d: int) -> Tuple[int, ...]:
        """Order in which the d regions of a level are interpolated.

        Per-level: fastest-varying axis first (Section VI-C, "fastest direction
        interpolation").  Per-region: the tuned permutation (Section IV).
        """
        if self.kind == "level" or self.order is None:
            return tuple(range(d - 1, -1, -1))
        order = tuple(int(a) for a in self.order)
        assert sorted(order) == list(range(d)), "order must be a permutation of the axes"
        return order


@dataclass(frozen=True)
class Target:
    """Retrieval target.

    kind: "abs"  absolute max error bound tau
          "rel"  tau = value * (max x - min x)
          "psnr" PSNR target in dB (Section III-A definition)
          "rmse" absolute RMSE bound (the PSNR mode's internal form)
    """
    kind: str
    value: float
