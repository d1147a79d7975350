"""Seeded synthetic CIELAB images for the GMM superpixel EM.

This package only makes inputs. It holds none of the method's arithmetic and is
the one module that both the CPU oracle side and the HIP side read from.
"""
from .voronoi_lab import (  # noqa: F401
    VoronoiImage,
    voronoi_lab,
    voronoi_srgb8,
    config1_image,
    config2_image,
    config3_batch,
    config4_image,
    config5_batch,
    separated_blocks,
    BLOCK_PALETTE,
    pack_batch,
)
