"""Sizes and distributions of the five synthetic workloads.

The mechanisms stand in for the paper's hydrogen-air (9 species) and
GRI-3.0-sized hydrocarbon workloads (Sec. 4 and Sec. 5); only their sizes are
mirrored.  Configurations 2 and 4 reuse the mechanism of configuration 1.
"""

# kg/mol; standard atomic weights
ATOMIC_WEIGHTS = {"H": 1.008e-3, "C": 12.011e-3, "N": 14.007e-3,
                  "O": 15.999e-3, "Ar": 39.95e-3}

SEEDS = {
    "mechanism": 1000,   # + config index
    "states": 2000,      # + config index
    "vjp_weights": 3000,  # + config index
    "surrogate_train": 4000,
    "surrogate_heldout": 4001,
}

CONFIGS = {
    0: dict(
        name="h2air-shaped-9sp-21rxn",
        elements=("H", "O", "N"),
        bounds={"H": (0, 4), "O": (0, 2), "N": (0, 2)},
        max_atoms=6,
        n_species=9, n_reactions=21, n_irreversible=0,
        n_third_body=1, n_falloff=2,
        inert_argon=False,
        n_cells=4096,
        T_range=(800.0, 2500.0), log10p_range=None, p_fixed=101325.0,
        dirichlet_alpha=1.0,
    ),
    1: dict(
        name="ch4air-shaped-53sp-325rxn",
        elements=("C", "H", "O", "N", "Ar"),
        bounds={"C": (0, 2), "H": (0, 4), "O": (0, 2), "N": (0, 2)},
        max_atoms=6,
        n_species=53, n_reactions=325, n_irreversible=25,
        n_third_body=30, n_falloff=25,
        inert_argon=True,
        n_cells=1 << 22,
        T_range=(300.0, 3000.0), log10p_range=(4.0, 6.5), p_fixed=None,
        dirichlet_alpha=0.3,
    ),
    3: dict(
        name="hydrocarbon-shaped-160sp-900rxn",
        elements=("C", "H", "O", "N", "Ar"),
        # 102 compositions exist under the config-1 bounds, fewer than the 158
        # reacting species needed here, so larger molecules are allowed.
        bounds={"C": (0, 4), "H": (0, 9), "O": (0, 2), "N": (0, 2)},
        max_atoms=12,
        n_species=160, n_reactions=900, n_irreversible=0,
        n_third_body=60, n_falloff=40,
        inert_argon=True,
        n_cells=1 << 20,
        T_range=(300.0, 3000.0), log10p_range=(4.0, 6.5), p_fixed=None,
        dirichlet_alpha=0.3,
    ),
}

# workload-only configurations on top of the config-1 mechanism
CONFIGS[2] = dict(CONFIGS[1], name="ch4air-shaped-53sp-325rxn-vjp",
                  n_cells=1 << 20)
CONFIGS[4] = dict(CONFIGS[1], name="ch4air-shaped-53sp-325rxn-surrogate",
                  n_cells=1 << 22, n_train=1 << 24)


def mechanism_config(cfg: int) -> int:
    """Configuration whose mechanism file a workload uses."""
    return 1 if cfg in (2, 4) else cfg
