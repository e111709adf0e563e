"""Measured errors of the GPU parity tests.

Each test asserts its tolerance itself; record() also keeps the measured value so that a session can
write them out (FFX_ERROR_LOG=<path>, one JSON object per line) for the precision table of the design
notes: the complex64 error against the oracle on the complex64-rounded input (the kernel's arithmetic
error) and, where recorded, against the oracle on the original complex128 input (arithmetic plus input
rounding).
"""
import json

# amplitudes: absolute, no phase alignment; energies and gradients: relative to max(1, |reference|)
AMP = {"complex128": 1e-12, "complex64": 1e-5}
REL = {"complex128": 1e-12, "complex64": 1e-5}

RECORDS = []


def key(dtype) -> str:
    return str(dtype).replace("torch.", "")


def record(test: str, dtype, quantity: str, err: float, tol: float | None = None, **extra) -> float:
    RECORDS.append(dict(test=test, dtype=key(dtype), quantity=quantity, err=float(err), tol=tol, **extra))
    return float(err)


def dump(path: str) -> None:
    with open(path, "w") as f:
        for r in RECORDS:
            f.write(json.dumps(r) + "\n")
