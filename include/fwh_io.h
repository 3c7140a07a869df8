/*
 * fwh_io.h -- C ABI of the host-side readers (and writers) of the OpenCFD-FWH
 * input files: the control file, the surface geometry file, the observer file
 * and the per-step FW-H dataset (Sec. III A and Appendix A of Zhang, Yu, Liu,
 * Li, "An MPI-OpenMP mixing parallel open source FW-H code for aeroacoustics
 * calculation").  They fill the flat host arrays that fwh.h takes: geometry
 * y/normal [P][3], dS [P], observers [O][3], and time-major surface data
 * rho [N][P], u [3][N][P], p' [N][P].  Host code only; part of libfwh.so.
 *
 * File layouts.
 *  control.fwh (Appendix A1): a Fortran namelist, "&group key = value, ... /",
 *    "!" starts a comment.  Keys named in the text: Kstep_start, Kstep_end
 *    (first and last solver step used), delta_step (step interval between
 *    sampling frames) and FWH_data_Format (0 binary, 1 ASCII), plus Mach number,
 *    angle of attack, time step, number of observers, number of frames and
 *    OpenMP threads (Sec. III A), whose key names the text does not give.
 *  FWH_Surface_Geo.dat (Appendix A2, ASCII): a first text line
 *    "variables=x,y,z,n1,n2,n3,dS", the number of Faces, then for each Face its
 *    block dimensions "nx ny nz" (one of them 1) followed by nx*ny*nz subface
 *    lines "x y z n1 n2 n3 dS" (centre, unit outward normal, area).  Panels are
 *    numbered in file order across Faces.
 *  observers.dat (Sec. III A, ASCII): one observer "x y z" per line; blank lines
 *    are skipped.
 *  FWH-xxxxxxxx.dat (Appendix A3): one file per solver step, xxxxxxxx the step
 *    zero-padded to eight digits; the k-th sampling frame is step
 *    Kstep_start + k*delta_step.  The text gives no layout (its figure is
 *    missing); these readers take, per Face in the geometry file's order, the
 *    block dimensions then the density, the three velocity components and the
 *    pressure pulsation of each subface (nondimensional, as Sec. II D defines
 *    them):
 *      ASCII  (format 1): a line "nx ny nz", then one line "rho u1 u2 u3 p'" per
 *                         subface;
 *      binary (format 0): Fortran unformatted sequential records, each framed
 *                         by its byte length as a little-endian uint32 before
 *                         and after: per Face one record of three int32
 *                         dimensions, then one of 5*nx*ny*nz float64 values,
 *                         variable-major (all rho, all u1, u2, u3, then p').
 *
 * Ownership.  Every array belongs to the caller.  The *_read calls that size
 * their output take a capacity and can be called first with null arrays to
 * learn the counts.
 *
 * Threads.  fwh_io_frames_read reads frames concurrently on n_threads host
 * threads (0 = the hardware concurrency), one file per task; each task writes
 * only its own frame's rows.  The other calls run on the calling thread.
 *
 * Errors.  Every call returns FWH_IO_OK (0) or a negative code, and
 * fwh_io_last_error() returns a message for the calling thread's most recent
 * failure (file, line or record).  Nothing is thrown across the ABI and
 * nothing aborts.  On failure the contents of output arrays are unspecified.
 */
#ifndef FWH_IO_H
#define FWH_IO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FWH_IO_OK       0
#define FWH_IO_EINVAL  -1   /* null pointer, bad enum or count */
#define FWH_IO_ESIZE   -4   /* more entries than the capacity passed */
#define FWH_IO_EFILE   -8   /* a file cannot be opened, read or written */
#define FWH_IO_EFORMAT -9   /* the content does not follow the layout above */

/* dataset formats (the FWH_data_Format key) */
#define FWH_IO_BINARY 0
#define FWH_IO_ASCII  1

/* One namelist entry: group and key lower-cased, the value's text as written
 * (quotes kept, surrounding blanks and separating commas trimmed; an array
 * value keeps its commas). */
typedef struct fwh_io_kv {
    char group[64];
    char key[64];
    char value[192];
} fwh_io_kv;

/* Control file (Appendix A1).  Fills up to `cap` entries of kv (kv may be null
 * to count) and sets *n to the number of entries in the file.  FWH_IO_ESIZE if
 * there are more than cap; FWH_IO_EFORMAT for a key without "=" or an
 * unterminated string. */
int fwh_io_control_read(const char *path, fwh_io_kv *kv, int32_t cap, int32_t *n);

/* Geometry file (Appendix A2).  Sets *n_faces and *n_panels.  If y, normal and
 * dS are all non-null it fills y [P][3], normal [P][3], dS [P] (FWH_IO_ESIZE
 * beyond cap_panels); face_dims [F][3] (nx, ny, nz) is filled for the first
 * cap_faces Faces when non-null.  FWH_IO_EFORMAT for a missing count, a
 * dimension < 1 or a subface line without seven numbers. */
int fwh_io_geometry_read(const char *path, int64_t *n_faces, int64_t *n_panels, int64_t *face_dims, double *y,
                         double *normal, double *dS, int64_t cap_faces, int64_t cap_panels);

/* Writes a geometry file in the layout above (17 significant digits, so a
 * read returns the same doubles). */
int fwh_io_geometry_write(const char *path, int64_t n_faces, const int64_t *face_dims, const double *y,
                          const double *normal, const double *dS);

/* Observer file.  Sets *n_obs; fills x_obs [O][3] when non-null (FWH_IO_ESIZE
 * beyond cap).  FWH_IO_EFORMAT for a non-blank line without three numbers. */
int fwh_io_observers_read(const char *path, int64_t *n_obs, double *x_obs, int64_t cap);

/* Writes "dir/FWH-%08lld.dat" for `step` into out (cap bytes with the NUL). */
int fwh_io_frame_path(const char *dir, int64_t step, char *out, int64_t cap);

/* Reads the n_frames files of steps kstep_start + k*delta_step, k < n_frames,
 * from dir into row k of the time-major arrays rho [N][P], u [3][N][P],
 * pp [N][P] with N = n_frames, P = the panels of the n_faces Faces whose
 * dimensions face_dims [F][3] the geometry file gave.  out_dtype FWH_F64 (0)
 * stores double, FWH_F32 (1) float (rounded to nearest).  Every file must hold
 * exactly those Faces with those dimensions (FWH_IO_EFORMAT otherwise, as for
 * a short file, a bad record length or a missing number); FWH_IO_EFILE if a
 * file cannot be read.  The message names the failing file (the earliest among
 * those the threads reached). */
int fwh_io_frames_read(const char *dir, int64_t kstep_start, int64_t delta_step, int64_t n_frames, int32_t format,
                       int64_t n_faces, const int64_t *face_dims, int32_t out_dtype, void *rho, void *u, void *pp,
                       int32_t n_threads);

/* Writes one frame file in `format` from per-panel arrays of length P (the
 * panels of the n_faces Faces, file order).  ASCII values carry 17
 * significant digits, so a read returns the same doubles. */
int fwh_io_frame_write(const char *path, int32_t format, int64_t n_faces, const int64_t *face_dims,
                       const double *rho, const double *u1, const double *u2, const double *u3, const double *pp);

/* Message for the calling thread's most recent failure ("" after success). */
const char *fwh_io_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FWH_IO_H */
