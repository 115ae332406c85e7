"""Seeded synthetic inputs for the hyper-reduced RVE evaluation.

This package draws random numbers and arranges them into arrays. It holds none
of the method's arithmetic (no kinematics, no material law, no reduction), so
both the FP64 oracle and the GPU path can consume its arrays without sharing
any code of the method.
"""
from .generators import (  # noqa: F401
    THETA_REF,
    THETA_CONTRAST,
    MAT_J2,
    Cluster,
    make_cluster,
    make_cluster_illcond,
    make_macro_points,
    make_increments,
    make_load_path,
    make_snapshots,
    make_strain_field,
    init_indices,
    make_pod_snapshots,
    zipf_counts,
    perturbed_theta,
    WORKLOADS,
)
