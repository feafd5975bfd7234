"""Theoretical peak of a device in cell updates per second (Sec. III-B).

Eq. 4: Capability = Clock_Rate x Throughput x Lanes (x number of cores);
Eq. 5: Theo_peak = Capability / instructions per cell update, with 12 int32
instructions per cell (Alg. 1: five add/sub, six max, one move).

On CDNA4 (MI355X) a compute unit has four SIMDs that each retire 16 int32
lanes per clock, i.e. 64 int32 VALU lane-operations per clock per CU; the
MI355X has 256 CUs at a 2.4 GHz peak engine clock.  A packed 16-bit VALU
operation updates two cells per lane, doubling the ceiling.
"""
from __future__ import annotations

CELL_INSTRUCTIONS = 12
MI355X_CUS = 256
MI355X_CLOCK_MHZ = 2400
MI355X_LANE_OPS_PER_CLK_PER_CU = 64


def theo_peak_gcups(cores: int, lanes: int, throughput: float, clock_mhz: float,
                    instructions: int = CELL_INSTRUCTIONS) -> float:
    """Eq. 4-5 in GCUPS; ``throughput`` is instructions per lane per clock."""
    capability = clock_mhz * 1e6 * throughput * lanes * cores
    return capability / instructions / 1e9


def int_valu_lane_ops_per_s(cus: int = MI355X_CUS, clock_mhz: float = MI355X_CLOCK_MHZ) -> float:
    return cus * MI355X_LANE_OPS_PER_CLK_PER_CU * clock_mhz * 1e6


def mi355x_peak_gcups(cus: int = MI355X_CUS, clock_mhz: float = MI355X_CLOCK_MHZ,
                      cells_per_lane_op: int = 1) -> float:
    """MI355X by Eq. 5: 256 CU x 64 lanes/clk x 2.4 GHz / 12 = 3,276.8 GCUPS."""
    return int_valu_lane_ops_per_s(cus, clock_mhz) * cells_per_lane_op / CELL_INSTRUCTIONS / 1e9
