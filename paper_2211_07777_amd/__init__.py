"""fluxmi: Fourier-convolution Poisson / Biot-Savart solver for AMD MI355X (gfx950).

The compute path is the HIP library ``libfluxmi.so`` (C ABI, ``include/fluxmi.h``);
this package only marshals arguments (torch tensors for device memory and streams).
"""
from .fluxmi import (  # noqa: F401
    CELL, NODE, EVEN, ODD, PER, UNB, F64, F32, POISSON, BIOT_SAVART, BIOT_SAVART_FD2, BIOT_SAVART_FD4,
    BIOT_SAVART_FD6, CHAT2, CHAT2_VOL, HEJ2, HEJ4, HEJ6, HEJ8, HEJ10, HEJ0, LGF2,
    FluxmiError, Plan, Batch, Server, plan_inspect, solve_batched, batched_workspace_bytes, library,
    error_string,
)
