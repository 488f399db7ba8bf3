"""Seeded synthetic inputs shared by the tests, the benchmark and the CPU oracle.

This module holds no arithmetic of the solver method: it only draws the
per-column horizontal coefficients K_T and the right-hand sides f, and names
the five workloads.  Both the HIP path and the oracle receive these arrays as
plain inputs.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), used as a counter-based
generator: the n-th output (n = 0, 1, ...) of a stream started from state s0 is
mix(s0 + (n + 1) * GAMMA), with GAMMA = 0x9E3779B97F4A7C15 and the published
finaliser

    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    z =  z ^ (z >> 31)

Stream s of seed S starts from state S + s * 2**32.  Stream 0 draws K_T,
stream 1 + r draws right-hand side r, stream 2**31 draws the sizes of the
batched instances.  Values are generated in the canonical order
g = (j * nx + i) * nz + k (z-contiguous, the host order), so they do not depend
on the device layout.

Uniform U[0,1): (x >> 11) * 2**-53.  U[-1,1]: 2U - 1.  N(0,1): Box-Muller on the
pair (1 - U[2m], U[2m+1]), cos branch.
"""

from __future__ import annotations

import concurrent.futures
import dataclasses
import math
import os
import threading

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
# one-element arrays, not numpy scalars: scalar uint64 operands take a slow
# overflow-checked path
_M1 = np.array([0xBF58476D1CE4E5B9], dtype=np.uint64)
_M2 = np.array([0x94D049BB133111EB], dtype=np.uint64)
_G = np.array([GAMMA], dtype=np.uint64)
_S30, _S27, _S31, _S11 = (np.array([v], dtype=np.uint64) for v in (30, 27, 31, 11))
_MASK64 = (1 << 64) - 1
_CHUNK = 1 << 18

STREAM_KH = 0
STREAM_SIZES = 1 << 31


def stream_state(seed: int, stream: int) -> int:
    """Initial SplitMix64 state of stream `stream` for seed `seed`."""
    return (int(seed) + int(stream) * (1 << 32)) & _MASK64


def _workers() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _chunks(seed: int, stream: int, start: int, count: int, emit) -> None:
    """Run SplitMix64 over outputs start..start+count-1 in chunks, handing each
    uint64 chunk to emit(c0, c1, chunk).  Outputs are independent (counter
    based), so chunks run on a thread pool (numpy releases the GIL inside the
    ufuncs); emit must only touch its own slice [c0, c1)."""
    s0 = np.array([stream_state(seed, stream)], dtype=np.uint64)
    starts = list(range(0, count, _CHUNK))
    local = threading.local()

    def run(c0):
        c1 = min(count, c0 + _CHUNK)
        w = c1 - c0
        if getattr(local, "z", None) is None:
            m = max(1, min(count, _CHUNK))
            local.z = np.empty(m, dtype=np.uint64)
            local.t = np.empty(m, dtype=np.uint64)
        zz, tt = local.z[:w], local.t[:w]
        zz.view(np.int64)[:] = np.arange(start + c0 + 1, start + c1 + 1, dtype=np.int64)
        np.multiply(zz, _G, out=zz)
        np.add(zz, s0, out=zz)
        for shift, mul in ((_S30, _M1), (_S27, _M2)):
            np.right_shift(zz, shift, out=tt)
            np.bitwise_xor(zz, tt, out=zz)
            np.multiply(zz, mul, out=zz)
        np.right_shift(zz, _S31, out=tt)
        np.bitwise_xor(zz, tt, out=zz)
        emit(c0, c1, zz)

    nw = min(_workers(), len(starts))
    if nw <= 1:
        for c0 in starts:
            run(c0)
        return
    with concurrent.futures.ThreadPoolExecutor(max_workers=nw) as ex:
        for fut in [ex.submit(run, c0) for c0 in starts]:
            fut.result()


def splitmix64(seed: int, stream: int, start: int, count: int) -> np.ndarray:
    """Outputs start .. start+count-1 of the stream, as uint64."""
    out = np.empty(count, dtype=np.uint64)

    def emit(c0, c1, zz):
        out[c0:c1] = zz

    _chunks(seed, stream, start, count, emit)
    return out


def uniform01(seed: int, stream: int, count: int, start: int = 0, lo: float = 0.0,
              hi: float = 1.0) -> np.ndarray:
    """lo + (hi - lo) * U with U = (x >> 11) * 2**-53 (exact in float64)."""
    out = np.empty(count, dtype=np.float64)

    def emit(c0, c1, zz):
        np.right_shift(zz, _S11, out=zz)
        o = out[c0:c1]
        o[:] = zz.view(np.int64)
        o *= 2.0 ** -53
        if lo != 0.0 or hi != 1.0:
            o *= hi - lo
            o += lo

    _chunks(seed, stream, start, count, emit)
    return out


def uniform_pm1(seed: int, stream: int, count: int) -> np.ndarray:
    """2U - 1 (the scaling by 2 and shift by 1 are exact)."""
    return uniform01(seed, stream, count, lo=-1.0, hi=1.0)


def normal(seed: int, stream: int, count: int) -> np.ndarray:
    u = uniform01(seed, stream, 2 * count)
    u1 = 1.0 - u[0::2]
    u2 = u[1::2]
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)


# ---------------------------------------------------------------------------
# Coefficient and right-hand-side draws
# ---------------------------------------------------------------------------

def kh_constant(nx: int, ny: int, value: float = 1.0) -> np.ndarray:
    return np.full(nx * ny, float(value))


def kh_uniform(seed: int, nx: int, ny: int, lo: float = 0.5, hi: float = 2.0) -> np.ndarray:
    """Per-column K_T ~ U[lo, hi], canonical order j*nx + i."""
    return lo + (hi - lo) * uniform01(seed, STREAM_KH, nx * ny)


def kh_lognormal(seed: int, nx: int, ny: int, s: float = 0.5) -> np.ndarray:
    """Per-column K_T = exp(s * N(0,1)), canonical order j*nx + i."""
    return np.exp(s * normal(seed, STREAM_KH, nx * ny))


def rhs(seed: int, r: int, nx: int, ny: int, nz: int) -> np.ndarray:
    """Right-hand side number r, f ~ U[-1,1], canonical order (j*nx+i)*nz+k."""
    return uniform_pm1(seed, 1 + r, nx * ny * nz)


def quadratic_faces(nz: int) -> np.ndarray:
    """Vertical faces z_k = (k/nz)^2, k = 0..nz: finest at the bottom."""
    k = np.arange(nz + 1, dtype=np.float64)
    return (k / nz) ** 2


def uniform_faces(nz: int) -> np.ndarray:
    return np.arange(nz + 1, dtype=np.float64) / nz


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    nlevels: int
    kv: float
    sigma: float
    seed: int
    kh_model: str          # "const", "uniform", "lognormal"
    rtol: float
    nrhs: int = 1

    @property
    def unknowns(self) -> int:
        return self.nx * self.ny * self.nz

    def kh(self) -> np.ndarray:
        if self.kh_model == "const":
            return kh_constant(self.nx, self.ny)
        if self.kh_model == "uniform":
            return kh_uniform(self.seed, self.nx, self.ny)
        if self.kh_model == "lognormal":
            return kh_lognormal(self.seed, self.nx, self.ny)
        raise ValueError(self.kh_model)

    def zfaces(self) -> np.ndarray:
        return quadratic_faces(self.nz)

    def rhs(self, r: int = 0) -> np.ndarray:
        return rhs(self.seed, r, self.nx, self.ny, self.nz)


SMALL = Workload("periodic-64x64x64-kv1e3", 64, 64, 64, 4, 1e3, 1.0, 1, "const", 1e-5)
SHARE = Workload("periodic-1024x1024x128-kv1e4-Kuniform", 1024, 1024, 128, 6, 1e4, 1.0, 2,
                 "uniform", 1e-8)
LARGEST = Workload("periodic-2048x2048x128-kv1e5-Klognormal", 2048, 2048, 128, 7, 1e5, 1.0, 5,
                   "lognormal", 1e-8)


# ---------------------------------------------------------------------------
# The paper's flat-box model problem (robustness study)
# ---------------------------------------------------------------------------

# Depth of the atmosphere over the Earth's radius: H = D / R with D = 10 km
# and R = 6371 km (the paper only says H << 1).
FLAT_BOX_DEPTH = 10.0 / 6371.0


@dataclasses.dataclass(frozen=True)
class FlatBox:
    """-omega^2 (Lap_2D u + lambda^2 u_zz) + u = f on [0,1]^2 x [0,H]
    (Sec. 2.1.1): homogeneous Dirichlet side walls, Neumann top and bottom,
    equidistant layers, constant coefficients K = omega^2, K_v = omega^2
    lambda^2, with omega = nu_CFL h / 2 (eq. OmegaNumerical; nu_CFL = 8.4 in
    the paper's main runs, lambda -> 1 at high resolution)."""
    n: int
    nz: int
    nu: float
    nlevels: int
    ncoarse: int = 2
    lam: float = 1.0
    depth: float = FLAT_BOX_DEPTH
    seed: int = 7
    rtol: float = 1e-5      # five orders of magnitude, as in the paper's runs

    @property
    def name(self) -> str:
        return (f"flatbox-{self.n}x{self.n}x{self.nz}-nu{self.nu:g}-L{self.nlevels}"
                f"-nc{self.ncoarse}")

    @property
    def unknowns(self) -> int:
        return self.n * self.n * self.nz

    @property
    def K(self) -> float:
        return (0.5 * self.nu / self.n) ** 2

    @property
    def kv(self) -> float:
        return self.K * self.lam ** 2

    def kh(self) -> np.ndarray:
        return kh_constant(self.n, self.n, self.K)

    def zfaces(self) -> np.ndarray:
        return self.depth * uniform_faces(self.nz)

    def rhs(self, r: int = 0) -> np.ndarray:
        return rhs(self.seed, r, self.n, self.n, self.nz)

    def params(self) -> dict:
        """Keyword arguments shared by the library context and the oracle."""
        return dict(kv=self.kv, sigma=1.0, zfaces=self.zfaces(), kh=self.kh(), bc_h=1, bc_v=1,
                    ncoarse=self.ncoarse)


# CFL numbers of the robustness sweep, and the smoothing steps on the
# coarsest level the paper reports as sufficient for its 5-, 7- and 10-level
# hierarchies on 512^2 x 128 (Sec. 5.2): two up to nu = 16.8 for all three,
# then 30 / 5 / 2 at nu = 84 and 150 / 15 / 2 at nu = 840.
CFL_SWEEP = (2.1, 4.2, 8.4, 16.8, 84.0, 840.0)


def paper_coarse_sweeps(nlevels: int, nu: float) -> int:
    if nu <= 16.8 or nlevels >= 10:
        return 2
    table = {5: {84.0: 30, 840.0: 150}, 7: {84.0: 5, 840.0: 15}}
    return table.get(nlevels, {}).get(nu, 2)


def coarsen_levels(n: int, nmin: int = 32) -> int:
    """Levels for a batched instance: coarsen while the size stays >= nmin and even."""
    levels = 1
    while n % 2 == 0 and n // 2 >= nmin:
        n //= 2
        levels += 1
    return levels


def batched_instances(seed: int = 4, count: int = 64, nrhs: int = 4):
    """The batched workload: `count` instances with seeded sizes, 4 RHS each."""
    sizes = (128, 256, 384, 512)
    depths = (32, 64, 128)
    u = uniform01(seed, STREAM_SIZES, 2 * count)
    out = []
    for i in range(count):
        n = sizes[min(3, int(4.0 * u[2 * i]))]
        nz = depths[min(2, int(3.0 * u[2 * i + 1]))]
        out.append(Workload(f"batch{i}-{n}x{n}x{nz}", n, n, nz, coarsen_levels(n), 1e4, 1.0,
                            seed * 1000 + i, "uniform", 1e-8, nrhs))
    return out
