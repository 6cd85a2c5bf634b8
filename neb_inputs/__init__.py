"""Seeded synthetic inputs shared by the FP64 oracle and the GPU library.

This package only builds input data (triangle meshes, materials, lights,
cameras, deposit streams).  It holds none of the method's arithmetic: no
sampling, no intersection, no density estimation.  Both the oracle under
``oracle/`` and the HIP library consume what it produces.
"""
from .scenes import (  # noqa: F401
    MAT_DTYPE, LIGHT_DTYPE, CAM_DTYPE, Scene,
    MAT_LAMBERT, MAT_MIRROR, MAT_DIELECTRIC, MAT_GGX,
    tiny_box, room, city_block, city_lots, batch_rooms, box_room, furnace_sphere, disk_light_plane,
    point_light_plane,
    random_triangle_soup, deposit_stream, plane_deposits, sphere_deposits, query_points,
    scene_by_name,
)
