"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module draws scenes, cameras, dictionaries, text embeddings and target
feature maps.  It holds none of the splatting method's arithmetic: no
projection, binning, compositing, decoding or relevancy.  Both the oracle
(``oracle/``) and the HIP library consume exactly the float32 arrays it
returns.
"""
from .scenes import (  # noqa: F401
    Camera,
    Scene,
    CONFIGS,
    make_camera,
    orbit_camera,
    make_scene,
    make_text,
    make_target_factors,
    target_map,
    config_scene,
)
