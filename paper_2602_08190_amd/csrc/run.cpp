// Decode calls: from a device image, or transfer + decode pipelined over
// double-buffered staging slots (Sec. 3.3), and the completion / error call.
#include "plan.hpp"

namespace zf {

static void set_outputs(zf_plan_t *P, void *const *d_out, hipStream_t st) {
    const uint32_t n = uint32_t(P->cols.size());
    ZF_REQUIRE(d_out, ZF_E_INVALID, "null output table");
    for (uint32_t c = 0; c < n; c++) {
        const uint64_t need = P->cols[c]->view.plain_bytes;
        ZF_REQUIRE(d_out[c] || need == 0, ZF_E_INVALID, "output %u is null", c);
        ZF_REQUIRE((reinterpret_cast<uintptr_t>(d_out[c]) & 15u) == 0, ZF_E_INVALID,
                   "output %u is not 16-byte aligned", c);
    }
    ZF_HIP(launch_set_out_tab(P->d_out_tab, reinterpret_cast<uint8_t *const *>(d_out), n, P->d_scratch, st));
}

void decompress_async(zf_plan_t *P, const void *d_comp, uint64_t comp_bytes, void *const *d_out,
                      hipStream_t st) {
    ZF_REQUIRE(d_comp || P->image_bytes == 0, ZF_E_INVALID, "null device image");
    ZF_REQUIRE(comp_bytes >= P->image_bytes, ZF_E_TOO_SMALL, "device image holds %llu bytes, plan needs %llu",
               (unsigned long long)comp_bytes, (unsigned long long)P->image_bytes);
    set_outputs(P, d_out, st);
    LaunchArgs A = P->image_args;
    A.comp = static_cast<const uint8_t *>(d_comp);
    A.dict = static_cast<const uint8_t *>(d_comp);
    ZF_HIP(launch_decode(A, P->persistent_waves, P->waves_per_block, P->lz_blk, st,
                         P->profile ? &P->kind_ev : nullptr));
    if (P->profile) P->kinds_recorded = true;
    P->timing_valid = false;
}

void transfer_and_decompress(zf_plan_t *P, void *const *d_out, hipStream_t st, zf_timing *timing) {
    set_outputs(P, d_out, st);
    // copies start after everything already queued on `st` (including the
    // previous call's decodes, which read the same slots)
    ZF_HIP(hipEventRecord(P->ev_start, st));
    ZF_HIP(hipStreamWaitEvent(P->copy_stream, P->ev_start, 0));
    for (auto &cp : P->dict_copies)
        ZF_HIP(hipMemcpyAsync(P->d_dict + cp.dst_off, cp.src, cp.len, hipMemcpyHostToDevice, P->copy_stream));
    ZF_HIP(hipEventRecord(P->ev_dict, P->copy_stream));
    ZF_HIP(hipStreamWaitEvent(st, P->ev_dict, 0));
    const size_t ns = P->d_slots.size();
    for (size_t k = 0; k < P->batches.size(); k++) {
        Batch &b = P->batches[k];
        const int s = b.slot;
        if (k >= ns) ZF_HIP(hipStreamWaitEvent(P->copy_stream, P->slot_free[s], 0));
        ZF_HIP(hipEventRecord(P->ev_h2d0[k], P->copy_stream));
        for (auto &cp : b.copies)
            ZF_HIP(hipMemcpyAsync(P->d_slots[s] + cp.dst_off, cp.src, cp.len, hipMemcpyHostToDevice,
                                  P->copy_stream));
        ZF_HIP(hipEventRecord(P->ev_h2d1[k], P->copy_stream));
        ZF_HIP(hipEventRecord(P->slot_full[s], P->copy_stream));
        ZF_HIP(hipStreamWaitEvent(st, P->slot_full[s], 0));
        ZF_HIP(hipEventRecord(P->ev_dec0[k], st));
        if (b.exec) ZF_HIP(hipGraphLaunch(b.exec, st));
        else ZF_HIP(launch_decode(b.args, P->persistent_waves, P->waves_per_block, P->lz_blk, st));
        ZF_HIP(hipEventRecord(P->ev_dec1[k], st));
        ZF_HIP(hipEventRecord(P->slot_free[s], st));
    }
    ZF_HIP(hipEventRecord(P->ev_end, st));
    P->pending_timing = timing;
    P->timing_valid = true;
}

void sync_plan(zf_plan_t *P, hipStream_t st) {
    ZF_HIP(hipStreamSynchronize(st));
    ZF_HIP(hipStreamSynchronize(P->copy_stream));
    if (P->pending_timing && P->timing_valid) {
        zf_timing t{};
        float ms = 0;
        for (size_t k = 0; k < P->batches.size(); k++) {
            ZF_HIP(hipEventElapsedTime(&ms, P->ev_h2d0[k], P->ev_h2d1[k]));
            t.h2d_ms += ms;
            ZF_HIP(hipEventElapsedTime(&ms, P->ev_dec0[k], P->ev_dec1[k]));
            t.decode_ms += ms;
            t.comp_bytes += P->batches[k].w.comp_bytes;
            t.plain_bytes += P->batches[k].w.plain_bytes;
        }
        ZF_HIP(hipEventElapsedTime(&ms, P->ev_start, P->ev_end));
        t.wall_ms = ms;
        *P->pending_timing = t;
        P->pending_timing = nullptr;
    }
    uint32_t err = 0;
    ZF_HIP(hipMemcpy(&err, P->d_err, sizeof err, hipMemcpyDeviceToHost));
    ZF_REQUIRE(err == 0, ZF_E_CORRUPT, "a kernel found a corrupt stream (error word 0x%x)", err);
}

void set_profile(zf_plan_t *P, bool on) {
    if (on && !P->kind_ev.e0[0]) {
        for (uint32_t k = 0; k <= K_COUNT; k++) {
            ZF_HIP(hipEventCreate(&P->kind_ev.e0[k]));
            ZF_HIP(hipEventCreate(&P->kind_ev.e1[k]));
        }
    }
    P->profile = on;
    P->kinds_recorded = false;
}

void kind_ms(zf_plan_t *P, double *ms) {
    ZF_REQUIRE(P->kinds_recorded, ZF_E_STATE, "no profiled zf_decompress_async since profiling was switched on");
    for (uint32_t k = 0; k <= K_COUNT; k++) {
        ms[k] = -1.0;
        if (!P->kind_ev.used[k]) continue;
        ZF_HIP(hipEventSynchronize(P->kind_ev.e1[k]));
        float t = 0;
        ZF_HIP(hipEventElapsedTime(&t, P->kind_ev.e0[k], P->kind_ev.e1[k]));
        ms[k] = t;
    }
}

void clear_error(zf_plan_t *P) { (void)hipMemset(P->d_err, 0, sizeof(uint32_t)); }

}  // namespace zf
