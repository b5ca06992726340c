"""Helpers shared by the GPU parity tests (kernel schedules to force)."""
import pytest  # noqa: F401


def schedule_cases(prec, tile_max):
    """Kernel schedules forced one field at a time from the library's
    defaults, plus the combination the tuner picks on the benchmark star
    (single precision).  tile_max: the largest fused column tile the
    lattice's LDS allows."""
    from paper_1509_05063_amd import binding
    cases = [("default", {})]
    if prec == binding.LS_C64:
        cases += [(f"csr{v}", dict(csr_variant=v)) for v in (0, 1, 2)]
        cases += [(f"near{v}", dict(near_variant=v)) for v in (0, 1, 2, 3, 4)]
    for fv in (0, 1):
        for tc in sorted({1, 4, tile_max}):
            cases.append((f"fft{fv}-tile{tc}", dict(fft_variant=fv, fft_col_tile=tc)))
    cases += [(f"rows{n}", dict(fft_row_threads=n)) for n in (256, 512, 1024)]
    cases += [(f"rows{n}-inplace", dict(fft_row_threads=n, fft_rows_inplace=1)) for n in (256, 1024)]
    cases.append(("rows-first", dict(near_rows_first=1)))
    cases += [(f"cols{n}", dict(fft_variant=1, fft_col_threads=n, fft_col_tile=min(4, tile_max))) for n in (256, 512)]
    if prec == binding.LS_C64:
        cases.append(("star-tuned", dict(csr_variant=2, near_variant=3, fft_variant=1, fft_col_tile=min(4, tile_max),
                                         fft_row_threads=512, fft_col_threads=512)))
    return cases


def fused_tile_max(op, prec):
    """Largest fused column tile ls_set_schedule accepts (LDS limit)."""
    from paper_1509_05063_amd import binding
    best = 1
    for tc in (2, 4, 6, 8, 12, 16, 32):
        try:
            op.set_schedule(prec, fft_variant=1, fft_col_tile=tc)
            best = tc
        except binding.LSError:
            break
    return best
