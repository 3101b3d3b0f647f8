"""Seeded synthetic workloads shared by the tests, the smoke check and the bench.

This module holds only workload definitions (process names, energies, masses, sizes,
seeds); no part of the matrix-element arithmetic.  The momenta themselves come from
RAMBO with these parameters.
"""
M_TOP = 173.0
ALPHA_EM = 1.0 / 132.507
ALPHA_S = 0.118
PARAMS = (M_TOP, ALPHA_EM, ALPHA_S)

# name -> (final-state masses, sqrt(s) [GeV], events of the configuration at seed 0)
PROCESSES = {
    "ee_mumu": ((0.0, 0.0), 500.0, 8192),
    "gg_tt": ((M_TOP, M_TOP), 1500.0, 1 << 19),
    "gg_ttg": ((M_TOP, M_TOP, 0.0), 1500.0, 1 << 20),
    "gg_ttgg": ((M_TOP, M_TOP, 0.0, 0.0), 1500.0, 1 << 19),
    "gg_ttggg": ((M_TOP, M_TOP, 0.0, 0.0, 0.0), 1500.0, 1 << 18),
    "gg_gg": ((0.0, 0.0), 1500.0, 0),
    "ee_mumu_z": ((0.0, 0.0), 500.0, 8192),
}
QCD = ["gg_tt", "gg_ttg", "gg_ttgg", "gg_ttggg"]
ALL = ["ee_mumu"] + QCD
SEED = 0
HELICITY_FILTER_SEED = 0x5EED
HELICITY_FILTER_EVENTS = 1024


def n_par(name):
    return len(PROCESSES[name][0]) + 2


def final_masses(name):
    return PROCESSES[name][0]


def sqrt_s(name):
    return PROCESSES[name][1]
