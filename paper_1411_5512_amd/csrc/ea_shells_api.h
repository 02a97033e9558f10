// ea_shells_api.h -- full-vector C4 shells (eq. 3 over every displacement)
// of the batched form's published configurations and of the multispin-coded
// batch's samples (ea_batch_c4_shells, ea_msc_c4_shells in ea.h).
#pragma once

namespace {

// Sum the shells from the dense rows (FFT route for L = 2^k or 3 2^k unless
// ea_set_shell_route says otherwise, else the rows kernel), copy them to the
// host and wait.
ea_status shells_to_host(const unsigned long long *qd, int dw, unsigned long long *shells, void *fft_work, int L,
                         int n_shells, int64_t *out, hipStream_t stream)
{
    const bool fft = fft_work != nullptr;
    ea_status st = fft ? launch_fft_shells(qd, dw, L, n_shells, shells, fft_work, stream)
                       : launch_shell_rows(qd, L, n_shells, shells, stream);
    if (st != EA_OK) return st;
    EA_HIP(hipMemcpyAsync(out, shells, 8 * (size_t)n_shells, hipMemcpyDeviceToHost, stream));
    if (fft) return fft_shells_check(fft_work, L, stream);
    EA_HIP(hipStreamSynchronize(stream));
    return EA_OK;
}

// The call's scratch in the handle's buffer: the dense rows, the shells and
// (FFT route) the complex array; the shells zeroed on `stream`.
ea_status shell_scratch(ShellScratch &sc, int L, int n_shells, unsigned long long **qd, unsigned long long **shells,
                        void **fft_work, int *dw, hipStream_t stream)
{
    *dw = 2 * ((L + 63) / 64);
    const size_t q_words = (size_t)L * L * (size_t)*dw;
    const size_t fft_bytes = shells_by_fft(L) ? fft_work_bytes(L) : 0;
    const size_t words = q_words + (size_t)n_shells, head = (8 * words + 255) / 256 * 256;
    ea_status st = sc.reserve(head + fft_bytes);
    if (st != EA_OK) return st;
    unsigned long long *base = (unsigned long long *)sc.p;
    *qd = base;
    *shells = base + q_words;
    *fft_work = fft_bytes ? (void *)((char *)sc.p + head) : nullptr;
    hipLaunchKernelGGL(ea::zero_u64_kernel, dim3(blocks_for((size_t)n_shells)), dim3(256), 0, stream, *shells,
                       (size_t)n_shells);
    EA_HIP(hipGetLastError());
    return EA_OK;
}

}  // namespace

extern "C" {

ea_status ea_batch_c4_shells(ea_batch *b, int32_t job, int32_t k, int32_t n_shells, int64_t *out)
{
    if (!b || !out) return fail(EA_ERR_ARG, "NULL argument");
    if (job < 0 || job >= (int32_t)b->jobs.size()) return fail(EA_ERR_ARG, "job %d out of range", job);
    const BatchJobHost &h = b->jobs[(size_t)job];
    if (k < 0 || k >= h.job.n_meas) return fail(EA_ERR_ARG, "measurement %d out of range", k);
    if (h.meas_t[(size_t)k] > h.t_host || !h.started)
        return fail(EA_ERR_STATE, "measurement %d (t=%u) not reached", k, h.meas_t[(size_t)k]);
    const int L = h.job.L;
    const int max_shells = 3 * (L / 2) * (L / 2) + 1;
    if (n_shells < 1 || n_shells > max_shells)
        return fail(EA_ERR_ARG, "n_shells=%d outside [1, %d]", n_shells, max_shells);
    unsigned long long *qd = nullptr, *shells = nullptr;
    void *fft_work = nullptr;
    int dw = 0;
    ea_status st = shell_scratch(b->shell_scratch, L, n_shells, &qd, &shells, &fft_work, &dw, b->stream);
    if (st != EA_OK) return st;
    // the configuration published at measurement k: [replica][colour][POS]
    ea::Lattice lat{};
    lat.spins = (uint32_t *)(h.base + h.off_mspins) + (size_t)k * 4 * (size_t)h.POS;
    ea::Geom g{};
    g.L = L;
    g.R = L / 2;
    g.RW = h.RW;
    g.rows = L * L;
    g.plane = h.POS;
    const size_t q_words = (size_t)L * L * (size_t)dw;
    EA_DISPATCH_W(h.W, hipLaunchKernelGGL((ea::dense_q_kernel<WW>), dim3(blocks_for(q_words)), dim3(256), 0,
                                          b->stream, lat, g, dw, qd));
    EA_HIP(hipGetLastError());
    return shells_to_host(qd, dw, shells, fft_work, L, n_shells, out, b->stream);
}

ea_status ea_msc_c4_shells(ea_msc *m, int32_t sample, int32_t n_shells, int64_t *out)
{
    if (!m || !out) return fail(EA_ERR_ARG, "NULL argument");
    if (sample < 0 || sample >= m->B) return fail(EA_ERR_ARG, "sample %d outside [0, %d)", sample, m->B);
    const int L = m->L;
    const int max_shells = 3 * (L / 2) * (L / 2) + 1;
    if (n_shells < 1 || n_shells > max_shells)
        return fail(EA_ERR_ARG, "n_shells=%d outside [1, %d]", n_shells, max_shells);
    unsigned long long *qd = nullptr, *shells = nullptr;
    void *fft_work = nullptr;
    int dw = 0;
    ea_status st = shell_scratch(m->shell_scratch, L, n_shells, &qd, &shells, &fft_work, &dw, m->stream);
    if (st != EA_OK) return st;
    const size_t q_words = (size_t)L * L * (size_t)dw;
    hipLaunchKernelGGL(ea::msc_dense_q_kernel, dim3(blocks_for(q_words)), dim3(256), 0, m->stream, m->lat, m->geom,
                       m->M, sample / m->M, sample % m->M, dw, qd);
    EA_HIP(hipGetLastError());
    return shells_to_host(qd, dw, shells, fft_work, L, n_shells, out, m->stream);
}

}  // extern "C"
