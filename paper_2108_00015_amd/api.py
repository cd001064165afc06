"""PyTorch-facing binding of the ConKer C ABI (include/conker.h).

Argument marshalling only: every step runs in the HIP library.  Tensors must
be CUDA (HIP) tensors on the context's device; the work is queued on the
current torch stream of that device (or the stream the context was created
with).  Errors from the library raise ConkerError with the library's message.
"""
from __future__ import annotations

import ctypes as ct
import dataclasses
from typing import Optional, Sequence, Tuple

import torch

from . import _lib

_DT = {torch.float32: _lib.F32, torch.float64: _lib.F64}
PRECISIONS = {"f64": _lib.MM_F64, "f32": _lib.MM_F32, "split_bf16": _lib.MM_SPLIT_BF16,
              "split_f16": _lib.MM_SPLIT_F16}


class ConkerError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (_lib.STATUS_NAMES.get(status, status), msg))
        self.status = status


def _check_outside(nout: torch.Tensor, allow_outside: bool):
    """Tracers outside the grid (or with a non-finite coordinate or weight) are
    dropped by the mapping and counted on the device; unless allowed, any such
    tracer is an error (this waits for the stream)."""
    if allow_outside:
        return
    cnt = [int(v) for v in nout.cpu().tolist()]
    if any(cnt):
        raise ConkerError(_lib.ERANGE, "tracers outside the grid or non-finite, per catalog: %s "
                          "(pass allow_outside=True to drop them)" % cnt)


TUNE_FIELDS = ("x_tile", "y_tile", "x_resident", "mm_kernel", "radius_batch", "axis_order", "radix")


def _tune_dict(t) -> dict:
    d = {k: int(getattr(t, k)) for k in TUNE_FIELDS}
    d["ms"] = float(t.ms)
    return d


@dataclasses.dataclass(frozen=True)
class Grid:
    """Grid of spacing `cell` whose cell (0, 0, 0) starts at `origin` (Sec. 2.2)."""
    dims: Tuple[int, int, int]
    origin: Tuple[float, float, float]
    cell: float

    @property
    def n_cells(self) -> int:
        return int(self.dims[0]) * int(self.dims[1]) * int(self.dims[2])

    def c(self) -> _lib.ConkerGrid:
        g = _lib.ConkerGrid()
        for k in range(3):
            g.dims[k] = int(self.dims[k])
            g.origin[k] = float(self.origin[k])
        g.cell = float(self.cell)
        return g


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ct.c_void_p(t.data_ptr())


def num_tuples(n_radii: int, n: int) -> int:
    return int(_lib.load().conker_num_tuples(int(n_radii), int(n)))


def shell_size(r_cells: float) -> int:
    out = ct.c_int64()
    st = _lib.load().conker_shell_size(float(r_cells), ct.byref(out))
    if st != _lib.OK:
        raise ConkerError(st, "shell radius %g cells" % r_cells)
    return int(out.value)


def kspec_elems(grid: Grid) -> int:
    g = grid.c()
    return int(_lib.load().conker_kspec_elems(ct.byref(g)))


class Context:
    """One library context bound to a device and a HIP stream."""

    def __init__(self, device: int = 0, stream: Optional[torch.cuda.Stream] = None,
                 workspace_max_bytes: int = 0):
        self.lib = _lib.load()
        self.device = int(device)
        h = ct.c_void_p()
        s = (stream if stream is not None else torch.cuda.current_stream(self.device)).cuda_stream
        st = self.lib.conker_create(ct.byref(h), self.device, ct.c_void_p(s), int(workspace_max_bytes))
        if st != _lib.OK:
            raise ConkerError(st, self.lib.conker_last_error(None).decode())
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.conker_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int):
        if st != _lib.OK:
            raise ConkerError(st, self.lib.conker_last_error(self.h).decode())

    def set_stream(self, stream: torch.cuda.Stream):
        self._check(self.lib.conker_set_stream(self.h, ct.c_void_p(stream.cuda_stream)))

    def synchronize(self):
        self._check(self.lib.conker_synchronize(self.h))

    def profile(self, enable: bool = True):
        """Start (or stop) per-launch event timing; drops earlier records."""
        self._check(self.lib.conker_profile_enable(self.h, 1 if enable else 0))

    def profile_read(self) -> dict:
        """{kind name: (launches, total ms)} for every kind with at least one launch."""
        out = {}
        k = 0
        while True:
            name = self.lib.conker_profile_kind_name(k)
            if name is None:
                break
            n = ct.c_int64()
            ms = ct.c_double()
            self._check(self.lib.conker_profile_read(self.h, k, ct.byref(n), ct.byref(ms)))
            if n.value:
                out[name.decode()] = (int(n.value), float(ms.value))
            k += 1
        return out

    def workspace_bytes(self) -> int:
        return int(self.lib.conker_workspace_bytes(self.h))

    # ---- mapping -----------------------------------------------------------
    def grid_assign(self, grid: Grid, pos: torch.Tensor, w: Optional[torch.Tensor], out: torch.Tensor,
                    wsum: Optional[torch.Tensor] = None, n_outside: Optional[torch.Tensor] = None):
        if pos.dtype != torch.float32 or pos.dim() != 2 or pos.shape[1] != 3:
            raise ValueError("positions must be float32 [N, 3]")
        if w is not None and (w.dtype != torch.float32 or w.numel() != pos.shape[0]):
            raise ValueError("weights must be float32 [N]")
        if out.dtype not in _DT or out.numel() != grid.n_cells:
            raise ValueError("grid tensor must be float32/float64 with dims cells")
        if wsum is not None and wsum.dtype != torch.float64:
            raise ValueError("wsum must be float64")
        if n_outside is not None and n_outside.dtype != torch.int64:
            raise ValueError("n_outside must be int64")
        g = grid.c()
        self._check(self.lib.conker_grid_assign(self.h, ct.byref(g), _ptr(pos), _ptr(w), int(pos.shape[0]),
                                                _DT[out.dtype], _ptr(out), _ptr(wsum), _ptr(n_outside)))

    def form_delta(self, grid: Grid, D: torch.Tensor, R: torch.Tensor, wsum_data: torch.Tensor,
                   wsum_rand: torch.Tensor, alpha: torch.Tensor):
        if D.dtype != R.dtype or D.numel() != grid.n_cells or R.numel() != grid.n_cells:
            raise ValueError("D and R must be grids of one dtype")
        g = grid.c()
        self._check(self.lib.conker_form_delta(self.h, ct.byref(g), _DT[D.dtype], _ptr(D), _ptr(R),
                                               _ptr(wsum_data), _ptr(wsum_rand), _ptr(alpha)))

    # ---- kernels -----------------------------------------------------------
    def make_shell_kernels(self, grid: Grid, radii: Sequence[float], dtype=torch.float32
                           ) -> Tuple[torch.Tensor, list]:
        nr = len(radii)
        kel = kspec_elems(grid)
        out = torch.empty((nr, kel), dtype=dtype, device="cuda:%d" % self.device)
        rad = (ct.c_double * nr)(*[float(r) for r in radii])
        sizes = (ct.c_int64 * nr)()
        g = grid.c()
        self._check(self.lib.conker_make_shell_kernels(self.h, ct.byref(g), rad, nr, _DT[dtype], _ptr(out),
                                                       sizes))
        return out, [int(s) for s in sizes]

    # ---- convolution -------------------------------------------------------
    def convolve_shells(self, grid: Grid, field_a: torch.Tensor, field_b: Optional[torch.Tensor],
                        kspec: torch.Tensor, maps_a: Optional[torch.Tensor] = None,
                        maps_b: Optional[torch.Tensor] = None):
        nr = int(kspec.shape[0])
        dt = field_a.dtype
        if kspec.dtype != dt or (field_b is not None and field_b.dtype != dt):
            raise ValueError("fields and kernel spectra must share a dtype")
        shape = (nr,) + tuple(int(d) for d in grid.dims)
        if maps_a is None:
            maps_a = torch.empty(shape, dtype=dt, device=field_a.device)
        if field_b is not None and maps_b is None:
            maps_b = torch.empty(shape, dtype=dt, device=field_a.device)
        g = grid.c()
        self._check(self.lib.conker_convolve_shells(self.h, ct.byref(g), _DT[dt], _ptr(field_a), _ptr(field_b),
                                                    _ptr(kspec), nr, _ptr(maps_a), _ptr(maps_b)))
        return maps_a, maps_b

    # ---- summation ---------------------------------------------------------
    def contract_npt(self, grid: Grid, field: torch.Tensor, maps: torch.Tensor, n: int,
                     precision: str = "f64", out: Optional[torch.Tensor] = None) -> torch.Tensor:
        nr = int(maps.shape[0])
        cnt = num_tuples(nr, n)
        if out is None:
            out = torch.empty(max(cnt, 0), dtype=torch.float64, device=field.device)
        g = grid.c()
        self._check(self.lib.conker_contract_npt(self.h, ct.byref(g), _DT[field.dtype], _ptr(field), _ptr(maps),
                                                 nr, int(n), PRECISIONS[precision], _ptr(out)))
        return out

    def convolve_contract(self, grid: Grid, field_a: torch.Tensor, field_b: Optional[torch.Tensor],
                          kspec: torch.Tensor, n: int, precision: str = "split_bf16",
                          out_a: Optional[torch.Tensor] = None, out_b: Optional[torch.Tensor] = None,
                          centre_a: Optional[torch.Tensor] = None, centre_b: Optional[torch.Tensor] = None):
        """Convolution + summation without returning the maps; returns (W_a, W_b).

        n = 2..5 and every precision of contract_npt: the fused kernel (maps never stored) where
        it applies (fused_supported), else the maps of the lines carrying field in the context's
        workspace.  With centre fields (cross-correlation), the maps of field_a are summed against
        centre_a (and likewise b)."""
        nr = int(kspec.shape[0])
        cnt = num_tuples(nr, n)
        if out_a is None:
            out_a = torch.empty(max(cnt, 0), dtype=torch.float64, device=field_a.device)
        if field_b is not None and out_b is None:
            out_b = torch.empty(max(cnt, 0), dtype=torch.float64, device=field_a.device)
        g = grid.c()
        if centre_a is None and centre_b is None:
            self._check(self.lib.conker_convolve_contract(self.h, ct.byref(g), _DT[field_a.dtype], _ptr(field_a),
                                                          _ptr(field_b), _ptr(kspec), nr, int(n),
                                                          PRECISIONS[precision], _ptr(out_a), _ptr(out_b)))
        else:
            self._check(self.lib.conker_convolve_contract_cross(
                self.h, ct.byref(g), _DT[field_a.dtype], _ptr(field_a), _ptr(field_b), _ptr(centre_a),
                _ptr(centre_b), _ptr(kspec), nr, int(n), PRECISIONS[precision], _ptr(out_a), _ptr(out_b)))
        return out_a, out_b

    def pair_spectral(self, grid: Grid, field_a: torch.Tensor, field_b: Optional[torch.Tensor],
                      kspec: torch.Tensor, cross: bool = True):
        """n = 2 sums from the spectra (Parseval): (W_aa, W_bb, W_ab), each [n_radii] float64
        (W_bb, W_ab None without field_b; W_ab None unless cross)."""
        nr = int(kspec.shape[0])
        dev = field_a.device
        aa = torch.empty(nr, dtype=torch.float64, device=dev)
        bb = torch.empty(nr, dtype=torch.float64, device=dev) if field_b is not None else None
        ab = torch.empty(nr, dtype=torch.float64, device=dev) if (field_b is not None and cross) else None
        g = grid.c()
        self._check(self.lib.conker_pair_spectral(self.h, ct.byref(g), _DT[field_a.dtype], _ptr(field_a),
                                                  _ptr(field_b), _ptr(kspec), nr, _ptr(aa), _ptr(bb), _ptr(ab)))
        return aa, bb, ab

    def delta_field(self, grid: Grid, D: torch.Tensor, R: torch.Tensor, alpha: Optional[torch.Tensor] = None,
                    out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """delta = (D - alpha R) / (alpha R), 0 where alpha R = 0 (Eq. densitycont)."""
        if D.dtype != R.dtype or D.numel() != grid.n_cells or R.numel() != grid.n_cells:
            raise ValueError("D / R shape or dtype mismatch")
        out = torch.empty_like(D) if out is None else out
        g = grid.c()
        self._check(self.lib.conker_delta_field(self.h, ct.byref(g), _DT[D.dtype], _ptr(D), _ptr(R), _ptr(alpha),
                                                _ptr(out)))
        return out

    def ratio_combined(self, W_delta: torch.Tensor, W_rand: torch.Tensor, alpha: torch.Tensor, n: int):
        """Regions combined (Eq. ksi3combined): W_delta, W_rand [n_regions, count], alpha [n_regions].
        Returns (xi, numerator, denominator)."""
        if W_delta.shape != W_rand.shape or W_delta.dim() != 2 or alpha.numel() != W_delta.shape[0]:
            raise ValueError("W_delta / W_rand must be [n_regions, count] and alpha [n_regions]")
        Wd, Wr, a = W_delta.contiguous(), W_rand.contiguous(), alpha.contiguous()
        cnt = int(Wd.shape[1])
        xi = torch.empty(cnt, dtype=torch.float64, device=Wd.device)
        num, den = torch.empty_like(xi), torch.empty_like(xi)
        self._check(self.lib.conker_ratio_combined(self.h, int(Wd.shape[0]), _ptr(Wd), _ptr(Wr), _ptr(a), int(n),
                                                   cnt, _ptr(xi), _ptr(num), _ptr(den)))
        return xi, num, den

    def map_ratio(self, grid: Grid, N: torch.Tensor, map_N: torch.Tensor, W_R2: torch.Tensor, alpha: torch.Tensor,
                  out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Per-cell W_0 W_1 / <B_0 B_1> of one radius (W_R2, alpha: device float64 scalars)."""
        out = torch.empty_like(N) if out is None else out
        g = grid.c()
        self._check(self.lib.conker_map_ratio(self.h, ct.byref(g), _DT[N.dtype], _ptr(N), _ptr(map_N), _ptr(W_R2),
                                              _ptr(alpha), _ptr(out)))
        return out

    def value_histogram(self, values: torch.Tensor, lo: float, hi: float, n_bins: int) -> torch.Tensor:
        """int64 [n_bins + 2]: equal bins of [lo, hi), then below lo, then at or above hi."""
        v = values.contiguous()
        counts = torch.empty(n_bins + 2, dtype=torch.int64, device=v.device)
        self._check(self.lib.conker_value_histogram(self.h, _DT[v.dtype], _ptr(v), int(v.numel()), float(lo),
                                                    float(hi), int(n_bins), _ptr(counts)))
        return counts

    # ---- survey front end ----------------------------------------------------
    def sky_to_cartesian(self, ra_deg: torch.Tensor, dec_deg: torch.Tensor, z: torch.Tensor,
                         cosmo: Optional["Cosmology"] = None) -> torch.Tensor:
        """float32 [n, 3] comoving positions from float64 ra, dec (degrees) and z."""
        cosmo = Cosmology() if cosmo is None else cosmo
        ra, dec, zz = (t.contiguous() for t in (ra_deg, dec_deg, z))
        if any(t.dtype != torch.float64 for t in (ra, dec, zz)) or not (ra.numel() == dec.numel() == zz.numel()):
            raise ValueError("ra, dec, z must be float64 of one length")
        pos = torch.empty((ra.numel(), 3), dtype=torch.float32, device=ra.device)
        cs = cosmo.c_struct()
        self._check(self.lib.conker_sky_to_cartesian(self.h, ct.byref(cs), _ptr(ra), _ptr(dec), _ptr(zz),
                                                     int(ra.numel()), _ptr(pos)))
        return pos

    def analytic_randoms(self, grid: Grid, n_tot: float, p_ang: torch.Tensor, ra_range, dec_range,
                         p_z: torch.Tensor, z_range, cosmo: Optional["Cosmology"] = None,
                         dtype=torch.float64) -> torch.Tensor:
        """Expected random count per cell from factorizable selection functions (Eq. factorizablility)."""
        cosmo = Cosmology() if cosmo is None else cosmo
        pa, pz = p_ang.contiguous(), p_z.contiguous()
        if pa.dtype != torch.float64 or pz.dtype != torch.float64 or pa.dim() != 2:
            raise ValueError("p_ang [n_dec, n_ra] and p_z [n_z] must be float64")
        R = torch.empty(tuple(int(d) for d in grid.dims), dtype=dtype, device=pa.device)
        g = grid.c()
        cs = cosmo.c_struct()
        rr = (ct.c_double * 2)(*ra_range)
        dr = (ct.c_double * 2)(*dec_range)
        zr = (ct.c_double * 2)(*z_range)
        self._check(self.lib.conker_analytic_randoms(self.h, ct.byref(g), _DT[dtype], ct.byref(cs), float(n_tot),
                                                     _ptr(pa), int(pa.shape[0]), int(pa.shape[1]), rr, dr, _ptr(pz),
                                                     int(pz.numel()), zr, _ptr(R)))
        return R

    def ratio_cross(self, Wc: torch.Tensor, Wr: torch.Tensor, alpha0: torch.Tensor, alpha1: torch.Tensor, n: int,
                    out: Optional[torch.Tensor] = None) -> torch.Tensor:
        out = torch.empty_like(Wc) if out is None else out
        self._check(self.lib.conker_ratio_cross(self.h, _ptr(Wc), _ptr(Wr), _ptr(alpha0), _ptr(alpha1), int(n),
                                                int(Wc.numel()), _ptr(out)))
        return out

    # ---- equidistant (diagonal) sums, Eq. ksinDiag ---------------------------
    def contract_diag(self, grid: Grid, field: torch.Tensor, maps: torch.Tensor, n_max: int) -> torch.Tensor:
        """[n_max - 1, n_radii] float64: row n - 2 holds sum_x field * maps[m]^(n-1)."""
        nr = int(maps.shape[0])
        if maps.dtype != field.dtype or maps.numel() != nr * grid.n_cells or field.numel() != grid.n_cells:
            raise ValueError("field / maps shape or dtype mismatch")
        out = torch.empty((n_max - 1, nr), dtype=torch.float64, device=field.device)
        g = grid.c()
        self._check(self.lib.conker_contract_diag(self.h, ct.byref(g), _DT[field.dtype], _ptr(field), _ptr(maps),
                                                  nr, int(n_max), _ptr(out)))
        return out

    def contract_diag_noalloc(self, grid: Grid, field: torch.Tensor, maps: torch.Tensor, n_max: int,
                              out: torch.Tensor) -> torch.Tensor:
        """contract_diag into a caller-given out ([n_max - 1, n_radii] float64): the library
        allocates nothing (conker_contract_diag_noalloc)."""
        nr = int(maps.shape[0])
        if maps.dtype != field.dtype or maps.numel() != nr * grid.n_cells or field.numel() != grid.n_cells:
            raise ValueError("field / maps shape or dtype mismatch")
        if out.dtype != torch.float64 or out.numel() != (n_max - 1) * nr:
            raise ValueError("out must be float64 with (n_max - 1) * n_radii values")
        g = grid.c()
        self._check(self.lib.conker_contract_diag_noalloc(self.h, ct.byref(g), _DT[field.dtype], _ptr(field),
                                                          _ptr(maps), nr, int(n_max), _ptr(out)))
        return out

    def convolve_diag(self, grid: Grid, field_a: torch.Tensor, field_b: Optional[torch.Tensor],
                      kspec: torch.Tensor, n_max: int, centre_a: Optional[torch.Tensor] = None,
                      centre_b: Optional[torch.Tensor] = None):
        """Diagonal sums of both fields without storing maps: (out_a, out_b), each [n_max - 1, n_radii].
        With centre fields the maps of field_a are summed against centre_a (cross-correlation)."""
        nr = int(kspec.shape[0])
        dt = field_a.dtype
        if kspec.dtype != dt or (field_b is not None and field_b.dtype != dt):
            raise ValueError("dtype mismatch")
        oa = torch.empty((n_max - 1, nr), dtype=torch.float64, device=field_a.device)
        ob = torch.empty_like(oa) if field_b is not None else None
        g = grid.c()
        if centre_a is None and centre_b is None:
            self._check(self.lib.conker_convolve_diag(self.h, ct.byref(g), _DT[dt], _ptr(field_a), _ptr(field_b),
                                                      _ptr(kspec), nr, int(n_max), _ptr(oa), _ptr(ob)))
        else:
            self._check(self.lib.conker_convolve_diag_cross(
                self.h, ct.byref(g), _DT[dt], _ptr(field_a), _ptr(field_b), _ptr(centre_a), _ptr(centre_b),
                _ptr(kspec), nr, int(n_max), _ptr(oa), _ptr(ob)))
        return oa, ob

    # ---- batches -----------------------------------------------------------
    def batch_plan(self, jobs):
        """Plans (and runs once, synchronously) a list of Job."""
        self._jobs = list(jobs)   # keep every tensor alive while the batch exists
        arr = (_lib.ConkerJob * len(self._jobs))(*[j.c() for j in self._jobs])
        self._check(self.lib.conker_batch_plan(self.h, ct.cast(arr, ct.c_void_p), len(self._jobs)))

    def batch_run(self):
        self._check(self.lib.conker_batch_run(self.h))

    def batch_capture(self):
        self._check(self.lib.conker_batch_capture(self.h))

    def batch_launch(self):
        self._check(self.lib.conker_batch_launch(self.h))

    def batch_classes(self, on: bool = True):
        """Whether later batch_plan calls run size classes of jobs stage by stage
        (the default) or every job alone."""
        self._check(self.lib.conker_batch_classes(self.h, 1 if on else 0))

    def batch_layout(self) -> list:
        """For each planned job, the chunk of a size class it runs in, or -1 (alone)."""
        jobs = getattr(self, "_jobs", [])
        arr = (ct.c_int * max(1, len(jobs)))()
        self._check(self.lib.conker_batch_layout(self.h, ct.cast(arr, ct.c_void_p)))
        return [int(arr[k]) for k in range(len(jobs))]

    def batch_autotune(self, reps: int = 3) -> list:
        """Times launch settings per job shape (after batch_plan) and keeps the
        fastest for later batch_run / batch_capture; returns one dict per job."""
        jobs = getattr(self, "_jobs", [])
        arr = (_lib.ConkerTune * len(jobs))()
        self._check(self.lib.conker_batch_autotune(self.h, int(reps), ct.cast(arr, ct.c_void_p) if jobs else None))
        return [_tune_dict(t) for t in arr]

    def set_tune(self, **fields):
        """Launch setting for later calls: x_tile, y_tile (1 narrow, 2 wide),
        x_resident (1 streamed, 2 resident with two LDS exchange buffers where
        they fit, 3 resident with one), mm_kernel (1 per-wave tiles,
        2 operand sharing, 3 n = 3 every tile per wave), radius_batch, axis_order (1 as given, 2..6 the
        other permutations of a cubic grid, see conker.h), radix (1 radix-8-first schedules, 2 radix 16
        first where that saves a stage); 0 or omitted = default."""
        bad = set(fields) - set(TUNE_FIELDS)
        if bad:
            raise ValueError("unknown launch setting(s): %s" % sorted(bad))
        t = _lib.ConkerTune(**{k: int(v) for k, v in fields.items()})
        self._check(self.lib.conker_set_tune(self.h, ct.byref(t)))

    def axis_order_used(self) -> int:
        """Axis order (1..6, see set_tune) of the last map-free summation; 0 if none ran."""
        v = ct.c_int()
        self._check(self.lib.conker_axis_order_used(self.h, ct.byref(v)))
        return int(v.value)

    AXIS_ORDERS = {1: (0, 1, 2), 2: (0, 2, 1), 3: (1, 0, 2), 4: (1, 2, 0), 5: (2, 0, 1), 6: (2, 1, 0)}

    def get_tune(self) -> dict:
        t = _lib.ConkerTune()
        self._check(self.lib.conker_get_tune(self.h, ct.byref(t)))
        return _tune_dict(t)

    def ratio(self, Wd: torch.Tensor, Wr: torch.Tensor, alpha: torch.Tensor, n: int,
              out: Optional[torch.Tensor] = None) -> torch.Tensor:
        if out is None:
            out = torch.empty_like(Wd)
        self._check(self.lib.conker_ratio(self.h, _ptr(Wd), _ptr(Wr), _ptr(alpha), int(n), int(Wd.numel()),
                                          _ptr(out)))
        return out


@dataclasses.dataclass
class Cosmology:
    """Fiducial cosmology of Eq. hubbleint (defaults: the paper's runs, Sec. 3)."""
    omega_m: float = 0.307
    omega_k: float = 0.0
    omega_lambda: float = 0.693
    h0: float = 100.0
    c: float = 300000.0
    z_max: float = 3.0

    def c_struct(self) -> _lib.ConkerCosmology:
        return _lib.ConkerCosmology(self.omega_m, self.omega_k, self.omega_lambda, self.h0, self.c, self.z_max)


@dataclasses.dataclass
class Job:
    """One catalog pair of a batch (see conker_job); holds its tensors alive."""
    grid: Grid
    kspec: torch.Tensor
    n: int
    precision: str
    data_pos: torch.Tensor
    rand_pos: torch.Tensor
    data_w: Optional[torch.Tensor]
    rand_w: Optional[torch.Tensor]
    N: torch.Tensor
    R: torch.Tensor
    maps_N: Optional[torch.Tensor]
    maps_R: Optional[torch.Tensor]
    wsum: torch.Tensor
    nout: torch.Tensor
    alpha: torch.Tensor
    W_delta: torch.Tensor
    W_rand: torch.Tensor
    xi: torch.Tensor

    def c(self) -> _lib.ConkerJob:
        j = _lib.ConkerJob()
        j.grid = self.grid.c()
        j.dtype = _DT[self.N.dtype]
        j.prec = PRECISIONS[self.precision]
        j.n = int(self.n)
        j.n_radii = int(self.kspec.shape[0])
        j.d_kspec = _ptr(self.kspec)
        j.d_data_pos, j.d_data_w, j.n_data = _ptr(self.data_pos), _ptr(self.data_w), int(self.data_pos.shape[0])
        j.d_rand_pos, j.d_rand_w, j.n_rand = _ptr(self.rand_pos), _ptr(self.rand_w), int(self.rand_pos.shape[0])
        j.d_N, j.d_R = _ptr(self.N), _ptr(self.R)
        j.d_maps_N, j.d_maps_R = _ptr(self.maps_N), _ptr(self.maps_R)
        j.d_wsum, j.d_n_outside, j.d_alpha = _ptr(self.wsum), _ptr(self.nout), _ptr(self.alpha)
        j.d_W_delta, j.d_W_rand, j.d_xi = _ptr(self.W_delta), _ptr(self.W_rand), _ptr(self.xi)
        return j


def make_job(grid: Grid, kspec: torch.Tensor, n: int, precision: str, data_pos: torch.Tensor,
             rand_pos: torch.Tensor, data_w: Optional[torch.Tensor] = None, rand_w: Optional[torch.Tensor] = None,
             N: Optional[torch.Tensor] = None, R: Optional[torch.Tensor] = None,
             maps_N: Optional[torch.Tensor] = None, maps_R: Optional[torch.Tensor] = None,
             fused: Optional[bool] = None) -> Job:
    """Builds a Job, allocating what is not given.  Grid and map tensors may be
    shared between jobs of one batch (they run in order); outputs are per job.
    fused=True gives the job no map buffers: the library keeps the maps it needs
    in its workspace (fused kernel, maps of carrying lines, or a size class's
    workspace).  Jobs that share no buffer can run as one size class."""
    dev, dt = kspec.device, kspec.dtype
    shape = tuple(int(d) for d in grid.dims)
    nr = int(kspec.shape[0])
    if fused is None:
        fused = fused_supported(grid, nr, n, precision, dt)
    N = torch.empty(shape, dtype=dt, device=dev) if N is None else N
    R = torch.empty(shape, dtype=dt, device=dev) if R is None else R
    if fused:
        maps_N = maps_R = None
    elif maps_N is None:
        maps_N = torch.empty((nr,) + shape, dtype=dt, device=dev)
        maps_R = torch.empty((nr,) + shape, dtype=dt, device=dev)
    else:   # shared buffers: at least n_radii * cells elements of the kernel dtype
        need = nr * grid.n_cells
        for m in (maps_N, maps_R):
            if m is None or m.dtype != dt or m.numel() < need or not m.is_contiguous():
                raise ValueError("maps_N / maps_R must be contiguous %s buffers of >= %d elements" % (dt, need))
    for t in (N, R):
        if t.dtype != dt or t.numel() < grid.n_cells or not t.is_contiguous():
            raise ValueError("N / R must be contiguous %s buffers of >= %d elements" % (dt, grid.n_cells))
    cnt = num_tuples(nr, n)
    z = lambda k, t: torch.zeros(k, dtype=t, device=dev)  # noqa: E731
    return Job(grid, kspec, n, precision, data_pos, rand_pos, data_w, rand_w, N, R, maps_N, maps_R,
               z(2, torch.float64), z(2, torch.int64), z(1, torch.float64), z(cnt, torch.float64),
               z(cnt, torch.float64), z(cnt, torch.float64))


def fused_supported(grid: Grid, n_radii: int, n: int, precision: str, dtype) -> bool:
    """Whether conker_convolve_contract runs its fused kernel here, which never stores the maps
    (else it keeps the maps of the carrying lines in the context's workspace)."""
    return (dtype == torch.float32 and precision in ("f32", "split_bf16") and n in (2, 3)
            and int(grid.dims[2]) == 512 and 1 <= n_radii <= 30)


def npcf_diag(ctx: Context, grid: Grid, data_pos: torch.Tensor, rand_pos: torch.Tensor, kspec: torch.Tensor,
              n_max: int, data_w: Optional[torch.Tensor] = None, rand_w: Optional[torch.Tensor] = None,
              dtype=torch.float64, allow_outside: bool = False) -> dict:
    """Equidistant n-point functions (Eq. ksinDiag) for n = 2 .. n_max without storing maps.

    Returns xi, W_delta and W_rand_raw as [n_max - 1, n_radii] float64 (row n - 2 is order n),
    and alpha."""
    dev = data_pos.device
    shape = tuple(int(d) for d in grid.dims)
    N = torch.zeros(shape, dtype=dtype, device=dev)
    R = torch.zeros(shape, dtype=dtype, device=dev)
    wsum = torch.zeros(2, dtype=torch.float64, device=dev)
    nout = torch.zeros(2, dtype=torch.int64, device=dev)
    alpha = torch.empty(1, dtype=torch.float64, device=dev)
    ctx.grid_assign(grid, data_pos, data_w, N, wsum[0:1], nout[0:1])
    ctx.grid_assign(grid, rand_pos, rand_w, R, wsum[1:2], nout[1:2])
    ctx.form_delta(grid, N, R, wsum[0:1], wsum[1:2], alpha)
    Wd, Wr = ctx.convolve_diag(grid, N, R, kspec, n_max)
    xi = torch.empty_like(Wd)
    for k in range(n_max - 1):
        ctx.ratio(Wd[k], Wr[k], alpha, k + 2, out=xi[k])
    _check_outside(nout, allow_outside)
    return dict(xi=xi, W_delta=Wd, W_rand_raw=Wr, alpha=alpha, n_outside=nout)


def npcf_pair2(ctx: Context, grid: Grid, data_pos: torch.Tensor, rand_pos: torch.Tensor, kspec: torch.Tensor,
               data_w: Optional[torch.Tensor] = None, rand_w: Optional[torch.Tensor] = None,
               dtype=torch.float64, allow_outside: bool = False) -> dict:
    """The 2pcf (Eq. ksi2_delta) with both sums taken in Fourier space (conker_pair_spectral):
    no inverse transform and no map.  Returns xi, W_delta, W_rand_raw ([n_radii] float64), alpha."""
    dev = data_pos.device
    shape = tuple(int(d) for d in grid.dims)
    N = torch.zeros(shape, dtype=dtype, device=dev)
    R = torch.zeros(shape, dtype=dtype, device=dev)
    wsum = torch.zeros(2, dtype=torch.float64, device=dev)
    nout = torch.zeros(2, dtype=torch.int64, device=dev)
    alpha = torch.empty(1, dtype=torch.float64, device=dev)
    ctx.grid_assign(grid, data_pos, data_w, N, wsum[0:1], nout[0:1])
    ctx.grid_assign(grid, rand_pos, rand_w, R, wsum[1:2], nout[1:2])
    ctx.form_delta(grid, N, R, wsum[0:1], wsum[1:2], alpha)
    Wd, Wr, _ = ctx.pair_spectral(grid, N, R, kspec, cross=False)
    xi = ctx.ratio(Wd, Wr, alpha, 2)
    _check_outside(nout, allow_outside)
    return dict(xi=xi, W_delta=Wd, W_rand_raw=Wr, alpha=alpha, n_outside=nout)


def npcf_continuous(ctx: Context, grid: Grid, D: torch.Tensor, R: torch.Tensor, kspec: torch.Tensor, n: int,
                    precision: str = "f64", alpha: Optional[torch.Tensor] = None, fused: Optional[bool] = None) -> dict:
    """Continuous tracers (Sec. 2.7): delta = (D - R) / R, then xi_n = sum_x delta prod_i (delta *** K_{a_i})
    (Eq. ksin_cont), with no further normalisation.  Returns xi (= W) and delta."""
    delta = ctx.delta_field(grid, D, R, alpha)
    if fused is None:
        fused = True
    if fused:
        xi, _ = ctx.convolve_contract(grid, delta, None, kspec, n, precision)
    else:
        maps, _ = ctx.convolve_shells(grid, delta, None, kspec)
        xi = ctx.contract_npt(grid, delta, maps, n, precision)
    return dict(xi=xi, delta=delta)


def npcf_cross(ctx: Context, grid: Grid, data0_pos: torch.Tensor, data1_pos: torch.Tensor, rand_pos: torch.Tensor,
               kspec: torch.Tensor, n: int, data0_w: Optional[torch.Tensor] = None,
               data1_w: Optional[torch.Tensor] = None, rand_w: Optional[torch.Tensor] = None,
               precision: str = "f64", dtype=torch.float64, fused: Optional[bool] = None,
               allow_outside: bool = False) -> dict:
    """Cross-correlation of tracer 0 (vertex 0) with tracer 1 (the shells), both background-subtracted
    against one random catalog (Sec. 2.8): xi = W_cross / (alpha0 alpha1^(n-1) W_rand_raw)."""
    dev = data0_pos.device
    shape = tuple(int(d) for d in grid.dims)
    N0 = torch.zeros(shape, dtype=dtype, device=dev)
    N1 = torch.zeros(shape, dtype=dtype, device=dev)
    R = torch.zeros(shape, dtype=dtype, device=dev)
    wsum = torch.zeros(3, dtype=torch.float64, device=dev)
    nout = torch.zeros(3, dtype=torch.int64, device=dev)
    alpha = torch.empty(2, dtype=torch.float64, device=dev)
    ctx.grid_assign(grid, data0_pos, data0_w, N0, wsum[0:1], nout[0:1])
    ctx.grid_assign(grid, data1_pos, data1_w, N1, wsum[1:2], nout[1:2])
    ctx.grid_assign(grid, rand_pos, rand_w, R, wsum[2:3], nout[2:3])
    ctx.form_delta(grid, N0, R, wsum[0:1], wsum[2:3], alpha[0:1])
    ctx.form_delta(grid, N1, R, wsum[1:2], wsum[2:3], alpha[1:2])
    if fused is None:
        fused = True
    if fused:
        # maps of N1 summed against N0; maps of R_raw summed against R_raw
        Wc, Wr = ctx.convolve_contract(grid, N1, R, kspec, n, precision, centre_a=N0, centre_b=R)
    else:
        maps1, mapsR = ctx.convolve_shells(grid, N1, R, kspec)
        Wc = ctx.contract_npt(grid, N0, maps1, n, precision)
        Wr = ctx.contract_npt(grid, R, mapsR, n, precision)
    xi = ctx.ratio_cross(Wc, Wr, alpha[0:1], alpha[1:2], n)
    _check_outside(nout, allow_outside)
    return dict(xi=xi, W_cross=Wc, W_rand_raw=Wr, alpha=alpha, n_outside=nout)


def npcf(ctx: Context, grid: Grid, data_pos: torch.Tensor, rand_pos: torch.Tensor, kspec: torch.Tensor,
         n: int, data_w: Optional[torch.Tensor] = None, rand_w: Optional[torch.Tensor] = None,
         precision: str = "f64", dtype=torch.float64, bufs: Optional[dict] = None,
         fused: Optional[bool] = None, field_at_a_time: bool = False, allow_outside: bool = False) -> dict:
    """Mapping -> convolution -> summation -> estimator, chaining the C ABI calls.

    `bufs` may hold preallocated tensors (keys: N, R, maps_N, maps_R, wsum, nout, alpha) that are
    reused across calls.  With `fused` (default, unless field_at_a_time) the convolution and
    summation run as one call, conker_convolve_contract: its fused kernel never stores the maps
    (fused_supported), otherwise it keeps the maps of the lines carrying field in the context's
    workspace.  With `field_at_a_time` (separate path) the maps of
    N and R are made and summed one field after the other in a single maps buffer (half the memory;
    each field's radii are paired in the transforms).  Returns xi, W_delta, W_rand_raw, alpha and
    the buffers (all on the GPU).  Tracers outside the grid raise ConkerError unless
    `allow_outside` (checking them waits for the stream).
    """
    if fused is None:
        fused = not field_at_a_time
    dev = data_pos.device
    b = {} if bufs is None else bufs
    shape = tuple(int(d) for d in grid.dims)
    nr = int(kspec.shape[0])
    if "N" not in b:
        b["N"] = torch.empty(shape, dtype=dtype, device=dev)
        b["R"] = torch.empty(shape, dtype=dtype, device=dev)
        b["wsum"] = torch.empty(2, dtype=torch.float64, device=dev)
        b["nout"] = torch.empty(2, dtype=torch.int64, device=dev)
        b["alpha"] = torch.empty(1, dtype=torch.float64, device=dev)
    b["N"].zero_()
    b["R"].zero_()
    b["wsum"].zero_()
    b["nout"].zero_()
    ctx.grid_assign(grid, data_pos, data_w, b["N"], b["wsum"][0:1], b["nout"][0:1])
    ctx.grid_assign(grid, rand_pos, rand_w, b["R"], b["wsum"][1:2], b["nout"][1:2])
    ctx.form_delta(grid, b["N"], b["R"], b["wsum"][0:1], b["wsum"][1:2], b["alpha"])
    if fused:
        Wd, Wr = ctx.convolve_contract(grid, b["N"], b["R"], kspec, n, precision)
    elif field_at_a_time:
        if "maps_N" not in b:
            b["maps_N"] = torch.empty((nr,) + shape, dtype=dtype, device=dev)
        ctx.convolve_shells(grid, b["N"], None, kspec, b["maps_N"])
        Wd = ctx.contract_npt(grid, b["N"], b["maps_N"], n, precision)
        ctx.convolve_shells(grid, b["R"], None, kspec, b["maps_N"])
        Wr = ctx.contract_npt(grid, b["R"], b["maps_N"], n, precision)
    else:
        if "maps_N" not in b:
            b["maps_N"] = torch.empty((nr,) + shape, dtype=dtype, device=dev)
            b["maps_R"] = torch.empty((nr,) + shape, dtype=dtype, device=dev)
        ctx.convolve_shells(grid, b["N"], b["R"], kspec, b["maps_N"], b["maps_R"])
        Wd = ctx.contract_npt(grid, b["N"], b["maps_N"], n, precision)
        Wr = ctx.contract_npt(grid, b["R"], b["maps_R"], n, precision)
    xi = ctx.ratio(Wd, Wr, b["alpha"], n)
    _check_outside(b["nout"], allow_outside)
    return dict(xi=xi, W_delta=Wd, W_rand_raw=Wr, alpha=b["alpha"], n_outside=b["nout"], bufs=b)
