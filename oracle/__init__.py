"""Plain FP64 CPU oracle for RGF / n-diagonal RGF / DDRGF selected inversion, the
lesser Green's function on the band and lead self-energies by decimation.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The GPU library never
calls it and shares no code with it; a product path that routes through here
would be a CPU fallback and is forbidden.
"""
from .rgf_oracle import (  # noqa: F401
    OpCounter,
    block_accessor,
    dense_matrix,
    dense_selected,
    ddrgf,
    domain_layout,
    grad_band,
    grad_onsite,
    gamma_of,
    nrgf,
    rgf,
    rgf_mixed_products,
    solve_energy,
    transmission,
    transmission_g11,
)
from .ext_precision import (  # noqa: F401
    lu_factor_ext,
    lu_solve_ext,
    lu_solve_right_ext,
    nrgf_ext,
    solve_energy_ext,
    transmission_ext,
)
from .keldysh import bond_current, density, dos, lesser, lesser_dense  # noqa: F401,E402
from .leads import lead_self_energies, lead_self_energy, surface_gf  # noqa: F401,E402
