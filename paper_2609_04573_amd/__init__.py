"""MI355X-native adaptive progressive compressor.

``refactor`` a float field into bitplane streams once (``refactor_batch`` for
many), then ``retrieve`` it (``retrieve_batch`` for many)
at any max-error bound or PSNR; ``select_pipeline`` picks the interpolation
scheme and coefficient-decomposition direction from a sample.  All work runs
in the HIP library ``libapc.so`` (see ``include/apc.h``).
"""
from .apc import (ApcError, BelowFloor, BlockSet, Handle, Ladder, Scheme, Server, Target, axis_norms,  # noqa: F401
                  check_serialized, deserialize, deserialize_host, refactor, refactor_batch, retrieve_batch,
                  select_pipeline, tile_override, tile_width, tune_tiles)
