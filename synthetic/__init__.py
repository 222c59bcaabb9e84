"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This package builds tight-binding hopping lists and k-point planes. It holds
none of the Wilson-loop arithmetic: no Bloch phases, no diagonalisation, no
overlaps. Both the FP64 oracle and the HIP library consume what it returns.
"""
from .models import (  # noqa: F401
    HopList,
    qwz,
    bhz,
    bbh,
    choti,
    ssh,
    bond_shift_1d,
    atomic,
    product_state_2d,
    supercell,
    bhz_disordered,
    bhz_vacancies,
    wannier_like,
    bhz_spin_diag,
    spinful_bbh,
    spinful_bbh_disordered,
    spinful_bbh_spin_diag,
    rotated_bhz,
    write_tb,
    write_centres,
    kplane,
    concat_hops,
    link_grid,
    SERVED_TYPES,
    served_types,
    served_model,
    uneven_systems,
)
